// Host side of libzm: argument checking, polar-grid geometry, resident
// tables, workspace layout and the C entry points declared in zm.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "stage_body.h"
#include "zm_internal.h"

namespace zm {

static thread_local std::string g_err;

int log_level() {
    static const int level = [] {
        const char* v = std::getenv("ZM_LOG");
        const int l = v ? std::atoi(v) : 0;
        return l < 0 ? 0 : (l > kLogDebug ? kLogDebug : l);
    }();
    return level;
}

void log_msg(int level, const char* fmt, ...) {
    if (level > log_level()) return;
    static const char* const kName[] = {"", "error", "info", "debug"};
    char line[1024];
    int n = std::snprintf(line, sizeof line, "zm: %s: ", kName[level]);
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(line + n, sizeof line - n - 1, fmt, ap);
    va_end(ap);
    std::strcat(line, "\n");
    std::fputs(line, stderr);  // one write per line, so lines of concurrent threads do not interleave
}

void set_error(const std::string& msg) {
    g_err = msg;
    log_msg(kLogError, "%s", msg.c_str());
}

zm_status fail(zm_status s, const std::string& msg) {
    set_error(msg);
    return s;
}

zm_status hip_fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? ZM_ENOMEM : ZM_EDEVICE;
}

bool polar_fft_supported(zm_dtype dt, int A, int A2);

static int pow2ceil(long v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// cos / sin(2 pi a / N), a = 0..N-1, N divisible by 8.  Only the first
// octant is evaluated; the rest follows by the exact symmetries
// (c, s) -> (s, c) about pi/4 and quarter-turn rotations, so samples a and
// a + N/4 are exact 90-degree rotations of each other.
static void unit_circle(int N, std::vector<double>& cs) {
    cs.assign(2 * (size_t)N, 0.0);
    const int q4 = N / 4;
    const long double two_pi = 6.283185307179586476925286766559L;
    for (int a = 0; a < N; ++a) {
        const int qd = a / q4, b = a % q4;
        double c, s;
        if (2 * b <= q4) {
            const long double t = two_pi * (long double)b / (long double)N;
            c = (double)cosl(t);
            s = (double)sinl(t);
        } else {
            const long double t = two_pi * (long double)(q4 - b) / (long double)N;
            c = (double)sinl(t);
            s = (double)cosl(t);
        }
        double cc = c, ss = s;
        switch (qd) {
            case 1: cc = -s; ss = c; break;
            case 2: cc = -c; ss = -s; break;
            case 3: cc = s; ss = -c; break;
            default: break;
        }
        cs[2 * (size_t)a] = cc;
        cs[2 * (size_t)a + 1] = ss;
    }
}

// Gauss-Legendre nodes / weights on [-1, 1] (Newton on P_N in long double).
static void gauss_legendre(int N, std::vector<double>& x, std::vector<double>& w) {
    x.assign(N, 0.0);
    w.assign(N, 0.0);
    const long double pi = 3.141592653589793238462643383279L;
    for (int i = 0; i < N; ++i) {
        long double z = cosl(pi * ((long double)i + 0.75L) / ((long double)N + 0.5L));
        long double dp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= N; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / (long double)k;
                p0 = p1;
                p1 = p2;
            }
            if (N == 1) { p1 = z; p0 = 1.0L; }
            dp = (long double)N * (z * p1 - p0) / (z * z - 1.0L);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= N; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / (long double)k;
                p0 = p1;
                p1 = p2;
            }
            if (N == 1) { p1 = z; p0 = 1.0L; }
            dp = (long double)N * (z * p1 - p0) / (z * z - 1.0L);
        }
        x[N - 1 - i] = (double)z;  // ascending
        w[N - 1 - i] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
    }
}

zm_status note_call(zm_plan_s* p, hipStream_t s, bool may_create) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return ZM_OK;
    std::lock_guard<std::mutex> lk(p->mu);
    hipEvent_t ev = nullptr;
    for (auto& d : p->done)
        if (d.first == s) ev = d.second;
    if (!ev) {
        // take over the slot of a stream whose last call has completed
        for (auto& d : p->done)
            if (hipEventQuery(d.second) == hipSuccess) {
                d.first = s;
                ev = d.second;
                break;
            }
    }
    if (!ev) {
        if (!may_create) return ZM_OK;
        ZM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        p->done.emplace_back(s, ev);
    }
    ZM_HIP(hipEventRecord(ev, s));
    return ZM_OK;
}

// The staged resample + FFT serves FP32-family plans with A = 4096 when the
// environment variable ZM_STAGED is "1" at plan creation (it is slower than
// the direct gather on MI355X as built; kept, tested, for the comparison).
constexpr int kStageThreads = 1024;
static bool stage_enabled() {
    const char* v = std::getenv("ZM_STAGED");
    return v && v[0] == '1' && v[1] == '\0';
}

// ---- Static scratch for zm_moments_static (callers that cannot allocate) ----
// The spectra workspace of zm_moments_static lives in this array; every
// device the library runs on holds its own copy until the process ends.  Its
// device address is looked up once per device (with that device current)
// when the first plan on the device is created; host code uses only that
// address, never the array's name (a host-side stand-in).
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {};

}  // namespace zm

static __device__ __align__(256) char scratch[zm::kStaticScratchBytes];

namespace zm {

// Device address of `scratch` on `device`, which must be the current device.
static zm_status scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxScratchDevices)
        return fail(ZM_EUNSUPPORTED, "static scratch: device ordinal beyond the supported range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return ZM_OK;
}

void add_batch_ref(zm_plan_s* p, int delta) {
    std::lock_guard<std::mutex> lk(p->mu);
    p->batch_refs += delta;
}

static void free_plan(zm_plan_s* p) {
    if (!p) return;
    for (auto& d : p->done) (void)hipEventDestroy(d.second);
    void* bufs[] = {p->d_spx, p->d_trig, p->d_tw, p->d_table, p->d_jac, p->d_thi,
                    p->d_tlo, p->d_rowscale, p->d_items, p->d_rowmap, p->d_stage_win, p->d_stage_rows};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

template <typename T>
static zm_status dev_alloc(T** ptr, size_t count, size_t* total) {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)ptr, count * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    *total += count * sizeof(T);
    return ZM_OK;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static size_t spectrum_bytes(const zm_plan_s* p, int batch) {
    const size_t el = p->dtype == ZM_F64 ? sizeof(double) : sizeof(float);
    return (size_t)batch * (size_t)(p->n_max + 1) * 2 * (size_t)p->Rp * el;
}

static size_t workspace_bytes(const zm_plan_s* p, int batch) {
    size_t b = align256(spectrum_bytes(p, batch));
    if (p->dtype == ZM_F16X2) b += align256((size_t)batch * sizeof(float));
    return b;
}

static bool moments_supported(const zm_plan_s* p) {
    return p->n_max <= kMaxMomentOrder && polar_fft_supported(p->dtype, p->A, p->A2);
}


}  // namespace zm

using namespace zm;

extern "C" {

int zm_num_moments(int n_max) {
    if (n_max < 0) return -1;
    const int h = n_max / 2;
    return (n_max % 2 == 0) ? (h + 1) * (h + 1) : (h + 1) * (h + 2);
}

int zm_index(int n, int m) {
    if (n < 0 || m < 0 || m > n || ((n - m) & 1)) return -1;
    return canon_index(n, m);
}

const char* zm_status_str(zm_status s) {
    switch (s) {
        case ZM_OK: return "ZM_OK";
        case ZM_EINVAL: return "ZM_EINVAL: invalid argument";
        case ZM_ENOMEM: return "ZM_ENOMEM: out of memory";
        case ZM_EDEVICE: return "ZM_EDEVICE: HIP runtime error";
        case ZM_EUNSUPPORTED: return "ZM_EUNSUPPORTED: unsupported configuration";
        case ZM_EBUSY: return "ZM_EBUSY: resource busy";
    }
    return "unknown zm_status";
}

const char* zm_last_error(void) { return g_err.c_str(); }

zm_status zm_plan_ex(const zm_plan_desc* d, zm_plan_t* out) {
    if (!d || !out) return fail(ZM_EINVAL, "null descriptor or output pointer");
    *out = nullptr;
    if (d->n_max < 0 || d->n_max > kMaxTableOrder)
        return fail(ZM_EINVAL, "n_max must be in [0, " + std::to_string(kMaxTableOrder) + "]");
    if (d->H < 2 || d->W < 2) return fail(ZM_EINVAL, "frame must be at least 2 x 2");
    if (d->dtype < ZM_F64 || d->dtype > ZM_F16X2) return fail(ZM_EINVAL, "unknown dtype");
    // the kernels address a frame's pixels by 32-bit offsets
    if ((long long)d->H * d->W * (d->dtype == ZM_F64 ? 8 : 4) >= (1LL << 31))
        return fail(ZM_EINVAL, "frame must be smaller than 2^31 bytes (H * W * element size)");
    if (d->rule != ZM_RING_MIDPOINT && d->rule != ZM_RING_GAUSS_LEGENDRE) return fail(ZM_EINVAL, "unknown ring rule");
    const int D = std::min(d->H, d->W);
    const int R = d->rings > 0 ? d->rings : D / 2;
    if (d->rings < 0 || R < 1 || R > kMaxRings) return fail(ZM_EINVAL, "rings must be in [1, 4096]");
    int A = d->angles;
    if (A == 0) {
        long need = std::max<long>(2L * d->n_max + 2, (long)std::ceil(M_PI * R));
        A = pow2ceil(std::max<long>(need, kMinAngles));
    }
    if (A < kMinAngles || A > kMaxAngles || (A & (A - 1)) != 0)
        return fail(ZM_EINVAL, "angles must be a power of two in [32, 4096]");
    if (A < 2 * d->n_max + 2) return fail(ZM_EINVAL, "angles must be >= 2 n_max + 2");

    int dev = d->device;
    if (dev < 0) {
        ZM_HIP(hipGetDevice(&dev));
    } else {
        int cnt = 0;
        ZM_HIP(hipGetDeviceCount(&cnt));
        if (dev >= cnt) return fail(ZM_EINVAL, "device ordinal out of range");
    }
    ZM_DEVICE(dev);

    zm_plan_s* p = new zm_plan_s();
    p->n_max = d->n_max;
    p->H = d->H;
    p->W = d->W;
    p->D = D;
    p->R = R;
    p->A = A;
    p->Rp = (R + kRingPad - 1) / kRingPad * kRingPad;
    p->M = d->n_max + 1;
    p->num_moments = zm_num_moments(d->n_max);
    p->A2 = std::max(16, pow2ceil(d->n_max + 1));
    p->NK = std::max(64, pow2ceil(2L * d->n_max + 2));
    p->dtype = d->dtype;
    p->neumann = d->neumann ? 1 : 0;
    p->rule = d->rule;
    p->device = dev;
    p->cx = 0.5 * (d->W - 1);
    p->cy = 0.5 * (d->H - 1);
    p->rpx = 0.5 * D;

    // ring nodes / weights of the radial quadrature of eq. (1)
    std::vector<double> spx(R);
    p->rho.resize(R);
    p->w.resize(R);
    if (d->rule == ZM_RING_MIDPOINT) {
        for (int r = 0; r < R; ++r) {
            p->rho[r] = (double)(2 * r + 1) / (double)(2 * R);
            p->w[r] = (double)(2 * r + 1) / (2.0 * (double)R * (double)R);
            spx[r] = (double)(2 * r + 1) * p->rpx / (double)(2 * R);
        }
    } else {
        std::vector<double> x, wg;
        gauss_legendre(R, x, wg);
        for (int r = 0; r < R; ++r) {
            p->rho[r] = 0.5 * (x[r] + 1.0);
            p->w[r] = 0.5 * wg[r] * p->rho[r];
            spx[r] = p->rho[r] * p->rpx;
        }
    }

    // projection layout: m blocks of K_m rows (n = m, m+2, ..), padded to 16
    p->blk_rows.resize(p->M);
    p->blk_toff.resize(p->M);
    int rows = 0;
    std::vector<int> rowmap;
    for (int m = 0; m <= p->n_max; ++m) {
        const int km = (p->n_max - m) / 2 + 1;
        const int padded = (km + kRowTile - 1) / kRowTile * kRowTile;
        p->blk_rows[m] = km;
        p->blk_toff[m] = rows;
        for (int j = 0; j < padded; ++j) {
            if (j < km) {
                rowmap.push_back(canon_index(m + 2 * j, m));
                rowmap.push_back(((m + 2 * j) << 16) | m);
            } else {
                rowmap.push_back(-1);
                rowmap.push_back(0);
            }
        }
        for (int r0 = 0; r0 < padded; r0 += 32) p->items.push_back(zm_item{m, r0, std::min(32, padded - r0), rows});
        rows += padded;
    }
    p->table_rows = rows;

    std::vector<double> trig, ck;
    unit_circle(A, trig);
    unit_circle(p->NK, ck);
    std::vector<double> ckc(p->NK);
    for (int k = 0; k < p->NK; ++k) ckc[k] = ck[2 * (size_t)k];

    zm_status st = ZM_OK;
    size_t total = 0;
    double *d_rho = nullptr, *d_w = nullptr, *d_ck = nullptr;
    auto cleanup_tmp = [&]() {
        if (d_rho) (void)hipFree(d_rho);
        if (d_w) (void)hipFree(d_w);
        if (d_ck) (void)hipFree(d_ck);
    };
#define ZM_TRY(expr)                 \
    do {                             \
        st = (expr);                 \
        if (st != ZM_OK) {           \
            cleanup_tmp();           \
            free_plan(p);            \
            return st;               \
        }                            \
    } while (0)
#define ZM_TRYHIP(call)                          \
    do {                                         \
        hipError_t e_ = (call);                  \
        if (e_ != hipSuccess) ZM_TRY(hip_fail(e_, #call)); \
    } while (0)

    size_t tmp_bytes = 0;
    ZM_TRY(dev_alloc(&d_rho, R, &tmp_bytes));
    ZM_TRY(dev_alloc(&d_w, R, &tmp_bytes));
    ZM_TRY(dev_alloc(&d_ck, p->NK, &tmp_bytes));
    ZM_TRY(dev_alloc(&p->d_spx, R, &total));
    ZM_TRY(dev_alloc(&p->d_trig, 2 * (size_t)A, &total));
    ZM_TRY(dev_alloc(&p->d_table, (size_t)p->num_moments * R, &total));
    ZM_TRY(dev_alloc(&p->d_jac, 3 * (size_t)p->num_moments, &total));
    const bool with_moments = moments_supported(p);
    if (with_moments) {
        const size_t n = (size_t)p->table_rows * p->Rp;
        if (p->dtype == ZM_F64) {
            double* t;
            ZM_TRY(dev_alloc(&t, n, &total));
            p->d_thi = t;
            double* tw;
            ZM_TRY(dev_alloc(&tw, 2 * (size_t)A, &total));
            p->d_tw = tw;
        } else {
            if (p->dtype == ZM_F32) {
                float* t;
                ZM_TRY(dev_alloc(&t, n, &total));
                p->d_thi = t;
            } else {
                uint16_t *th, *tl;
                ZM_TRY(dev_alloc(&th, n, &total));
                ZM_TRY(dev_alloc(&tl, n, &total));
                p->d_thi = th;
                p->d_tlo = tl;
                if (p->dtype == ZM_F16X2) ZM_TRY(dev_alloc(&p->d_rowscale, (size_t)p->table_rows, &total));
            }
            float* tw;
            ZM_TRY(dev_alloc(&tw, 2 * (size_t)A, &total));
            p->d_tw = tw;
        }
        ZM_TRY(dev_alloc(&p->d_items, p->items.size(), &total));
        ZM_TRY(dev_alloc(&p->d_rowmap, rowmap.size(), &total));
    }

    ZM_TRYHIP(hipMemcpy(d_rho, p->rho.data(), R * sizeof(double), hipMemcpyHostToDevice));
    ZM_TRYHIP(hipMemcpy(d_w, p->w.data(), R * sizeof(double), hipMemcpyHostToDevice));
    ZM_TRYHIP(hipMemcpy(d_ck, ckc.data(), p->NK * sizeof(double), hipMemcpyHostToDevice));
    ZM_TRYHIP(hipMemcpy(p->d_spx, spx.data(), R * sizeof(double), hipMemcpyHostToDevice));
    ZM_TRYHIP(hipMemcpy(p->d_trig, trig.data(), 2 * (size_t)A * sizeof(double), hipMemcpyHostToDevice));
    {
        // Pixel-centre reconstruction: R_n^m(rho) = rho^m Q_k(x), x = 1 - 2 rho^2,
        // k = (n - m) / 2, Q_k = (-1)^k P_k^(m,0)(x) (Jacobi), by the three-term
        // recurrence Q_k = (alpha x + beta) Q_{k-1} + gamma Q_{k-2}, Q_0 = 1.
        // The coefficients depend on (k, m) only: one (alpha, beta, gamma) per moment.
        std::vector<double> jac(3 * (size_t)p->num_moments, 0.0);
        for (int n = 0; n <= p->n_max; ++n)
            for (int m = n & 1; m <= n; m += 2) {
                const int k = (n - m) / 2;
                const double kk = k, am = m;
                double al = 0.0, be = 0.0, ga = 0.0;
                if (k == 1) {
                    al = 0.5 * (am + 2.0);
                    be = 0.5 * am;
                } else if (k >= 2) {
                    const double a1 = 2.0 * kk * (kk + am) * (2.0 * kk + am - 2.0);
                    al = (2.0 * kk + am - 1.0) * (2.0 * kk + am) * (2.0 * kk + am - 2.0) / a1;
                    be = (2.0 * kk + am - 1.0) * am * am / a1;
                    ga = 2.0 * (kk + am - 1.0) * (kk - 1.0) * (2.0 * kk + am) / a1;
                }
                double* j = &jac[3 * (size_t)canon_index(n, m)];
                j[0] = -al;  // the (-1)^k of R_n^m folded into the recurrence
                j[1] = -be;
                j[2] = -ga;
            }
        ZM_TRYHIP(hipMemcpy(p->d_jac, jac.data(), jac.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if (with_moments) {
        if (p->dtype == ZM_F64) {
            ZM_TRYHIP(hipMemcpy(p->d_tw, trig.data(), 2 * (size_t)A * sizeof(double), hipMemcpyHostToDevice));
        } else {
            std::vector<float> twf(2 * (size_t)A);
            for (size_t i = 0; i < twf.size(); ++i) twf[i] = (float)trig[i];
            ZM_TRYHIP(hipMemcpy(p->d_tw, twf.data(), twf.size() * sizeof(float), hipMemcpyHostToDevice));
        }
        ZM_TRYHIP(hipMemcpy(p->d_items, p->items.data(), p->items.size() * sizeof(zm_item), hipMemcpyHostToDevice));
        ZM_TRYHIP(hipMemcpy(p->d_rowmap, rowmap.data(), rowmap.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    if (with_moments && p->dtype != ZM_F64 && p->A == 4096 && stage_enabled()) {
        std::vector<zmk::StageWin> wins;
        std::vector<int> rows;
        bool ok = false;
        switch (p->A2) {
            case 16: ok = zmk::stage_windows<4096, 16, kStageThreads>(p->H, p->W, p->R, p->Rp, p->cx, p->cy, spx, trig, wins, rows); break;
            case 32: ok = zmk::stage_windows<4096, 32, kStageThreads>(p->H, p->W, p->R, p->Rp, p->cx, p->cy, spx, trig, wins, rows); break;
            case 64: ok = zmk::stage_windows<4096, 64, kStageThreads>(p->H, p->W, p->R, p->Rp, p->cx, p->cy, spx, trig, wins, rows); break;
            case 128: ok = zmk::stage_windows<4096, 128, kStageThreads>(p->H, p->W, p->R, p->Rp, p->cx, p->cy, spx, trig, wins, rows); break;
            case 256: ok = zmk::stage_windows<4096, 256, kStageThreads>(p->H, p->W, p->R, p->Rp, p->cx, p->cy, spx, trig, wins, rows); break;
            default: break;
        }
        if (ok) {
            zmk::StageWin* dw = nullptr;
            ZM_TRY(dev_alloc(&dw, wins.size(), &total));
            p->d_stage_win = dw;
            ZM_TRY(dev_alloc(&p->d_stage_rows, rows.size(), &total));
            ZM_TRYHIP(hipMemcpy(dw, wins.data(), wins.size() * sizeof(zmk::StageWin), hipMemcpyHostToDevice));
            ZM_TRYHIP(hipMemcpy(p->d_stage_rows, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice));
            p->stage_nthr = kStageThreads;
        }
    }
    {
        hipError_t e = launch_zrp_table(p, d_rho, d_ck, nullptr);
        if (e != hipSuccess) ZM_TRY(hip_fail(e, "zrp_table kernel launch"));
        if (with_moments) {
            e = launch_fold(p, d_w, nullptr);
            if (e != hipSuccess) ZM_TRY(hip_fail(e, "fold kernel launch"));
        }
        e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) ZM_TRY(hip_fail(e, "plan construction"));
    }
    {
        // one completion event made up front (reused by calls that must not
        // allocate), and the static scratch's address on this device
        hipEvent_t ev = nullptr;
        ZM_TRYHIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        p->done.emplace_back(nullptr, ev);
        void* sp = nullptr;
        ZM_TRY(scratch_address(p->device, &sp));
    }
#undef ZM_TRY
#undef ZM_TRYHIP
    cleanup_tmp();
    p->resident = total;
    *out = p;
    log_msg(kLogInfo, "plan %p: n_max %d, %d x %d frames, %d rings (%d padded) x %d angles, dtype %d, %s rings, device %d, "
        "%zu resident bytes, %zu workspace bytes per frame", (void*)p, p->n_max, p->H, p->W, p->R, p->Rp, p->A,
        (int)p->dtype, p->rule == ZM_RING_GAUSS_LEGENDRE ? "Gauss-Legendre" : "midpoint", p->device, p->resident,
        workspace_bytes(p, 1) - workspace_bytes(p, 0));
    return ZM_OK;
}

zm_status zm_plan(int n_max, int H, int W, zm_dtype dtype, int neumann, zm_plan_t* out) {
    zm_plan_desc d;
    d.n_max = n_max;
    d.H = H;
    d.W = W;
    d.dtype = dtype;
    d.neumann = neumann;
    d.rings = 0;
    d.angles = 0;
    d.rule = ZM_RING_MIDPOINT;
    d.device = -1;
    return zm_plan_ex(&d, out);
}

zm_status zm_plan_info(zm_plan_t p, zm_plan_info_t* o) {
    if (!p || !o) return fail(ZM_EINVAL, "null plan or output");
    o->n_max = p->n_max;
    o->H = p->H;
    o->W = p->W;
    o->rings = p->R;
    o->angles = p->A;
    o->num_moments = p->num_moments;
    o->rings_padded = p->Rp;
    o->dtype = p->dtype;
    o->neumann = p->neumann;
    o->rule = p->rule;
    o->device = p->device;
    o->resident_bytes = p->resident;
    o->workspace_bytes_per_image = align256(spectrum_bytes(p, 1));
    o->workspace_bytes_fixed = p->dtype == ZM_F16X2 ? 256 : 0;
    return ZM_OK;
}

zm_status zm_radial_table(zm_plan_t p, double* host_out, size_t n_elems) {
    if (!p || !host_out) return fail(ZM_EINVAL, "null plan or output");
    const size_t need = (size_t)p->num_moments * p->R;
    if (n_elems < need) return fail(ZM_EINVAL, "output too small: need num_moments * rings elements");
    ZM_DEVICE(p->device);
    ZM_HIP(hipMemcpy(host_out, p->d_table, need * sizeof(double), hipMemcpyDeviceToHost));
    return ZM_OK;
}

zm_status zm_ring_nodes(zm_plan_t p, double* rho_out, double* w_out, size_t n_elems) {
    if (!p) return fail(ZM_EINVAL, "null plan");
    if (n_elems < (size_t)p->R) return fail(ZM_EINVAL, "output too small: need rings elements");
    if (rho_out) std::memcpy(rho_out, p->rho.data(), p->R * sizeof(double));
    if (w_out) std::memcpy(w_out, p->w.data(), p->R * sizeof(double));
    return ZM_OK;
}

zm_status zm_workspace_size(zm_plan_t p, int batch, size_t* bytes) {
    if (!p || !bytes) return fail(ZM_EINVAL, "null plan or output");
    if (batch < 0) return fail(ZM_EINVAL, "negative batch");
    *bytes = workspace_bytes(p, batch);
    return ZM_OK;
}

static zm_status check_run(zm_plan_t p, int batch, void* d_ws, size_t ws_bytes) {
    if (!p) return fail(ZM_EINVAL, "null plan");
    if (batch < 0) return fail(ZM_EINVAL, "negative batch");
    if (!moments_supported(p))
        return fail(ZM_EUNSUPPORTED, "moments need n_max <= 255 and angles <= 4096 (<= 1024 for ZM_F64)");
    if (batch == 0) return ZM_OK;
    if (batch > 65535) return fail(ZM_EINVAL, "batch must be <= 65535");
    if (!d_ws) return fail(ZM_EINVAL, "null workspace");
    const size_t need = workspace_bytes(p, batch);
    if (ws_bytes < need) return fail(ZM_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    return ZM_OK;
}

static float* fmax_slot(zm_plan_t p, void* d_ws, int batch) {
    return p->dtype == ZM_F16X2 ? (float*)((char*)d_ws + align256(spectrum_bytes(p, batch))) : nullptr;
}

static zm_status run_spectra(zm_plan_t p, const void* src, int batch, long long stride, void* d_ws,
                             size_t ws_bytes, zm_stream_t stream, int from_polar) {
    zm_status st = check_run(p, batch, d_ws, ws_bytes);
    if (st != ZM_OK || batch == 0) return st;
    if (!src) return fail(ZM_EINVAL, "null input pointer");
    ZM_DEVICE(p->device);
    hipStream_t s = (hipStream_t)stream;
    float* fmax = fmax_slot(p, d_ws, batch);
    if (fmax) {
        hipError_t e = launch_zero_u32((unsigned*)fmax, (size_t)batch, s);
        if (e != hipSuccess) return hip_fail(e, "zero kernel launch");
    }
    hipError_t e = launch_polar_fft(p, src, stride, batch, d_ws, fmax, from_polar, s);
    if (e != hipSuccess) return hip_fail(e, "resample+FFT kernel launch");
    return ZM_OK;
}

static zm_status run_project(zm_plan_t p, int batch, void* d_Z, void* d_ws, size_t ws_bytes, zm_stream_t stream) {
    zm_status st = check_run(p, batch, d_ws, ws_bytes);
    if (st != ZM_OK || batch == 0) return st;
    if (!d_Z) return fail(ZM_EINVAL, "null output pointer");
    ZM_DEVICE(p->device);
    hipError_t e = launch_project(p, d_ws, fmax_slot(p, d_ws, batch), batch, d_Z, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "projection kernel launch");
    return ZM_OK;
}

// Marks the completion of the call's work on the plan (for zm_destroy).
static zm_status noted(zm_status st, zm_plan_t p, int batch, zm_stream_t stream, const char* what) {
    if (st != ZM_OK || batch <= 0) return st;
    log_msg(kLogDebug, "%s: plan %p, batch %d, stream %p", what, (void*)p, batch, stream);
    ZM_DEVICE(p->device);
    return note_call(p, (hipStream_t)stream);
}

zm_status zm_spectra(zm_plan_t p, const void* d_images, int batch, long long image_stride, void* d_ws,
                     size_t ws_bytes, zm_stream_t stream) {
    if (p && batch > 1 && image_stride < (long long)p->H * p->W)
        return fail(ZM_EINVAL, "image_stride must be >= H * W");
    return noted(run_spectra(p, d_images, batch, image_stride, d_ws, ws_bytes, stream, 0), p, batch, stream,
                 "zm_spectra");
}

zm_status zm_project(zm_plan_t p, int batch, void* d_Z, void* d_ws, size_t ws_bytes, zm_stream_t stream) {
    return noted(run_project(p, batch, d_Z, d_ws, ws_bytes, stream), p, batch, stream, "zm_project");
}

zm_status zm_moments(zm_plan_t p, const void* d_images, int batch, long long image_stride, void* d_Z, void* d_ws,
                     size_t ws_bytes, zm_stream_t stream) {
    if (batch > 0 && !d_Z) return fail(ZM_EINVAL, "null output pointer");
    if (p && batch > 1 && image_stride < (long long)p->H * p->W)
        return fail(ZM_EINVAL, "image_stride must be >= H * W");
    zm_status st = run_spectra(p, d_images, batch, image_stride, d_ws, ws_bytes, stream, 0);
    if (st == ZM_OK) st = run_project(p, batch, d_Z, d_ws, ws_bytes, stream);
    return noted(st, p, batch, stream, "zm_moments");
}

zm_status zm_moments_polar(zm_plan_t p, const void* d_polar, int batch, void* d_Z, void* d_ws, size_t ws_bytes,
                           zm_stream_t stream) {
    if (!p) return fail(ZM_EINVAL, "null plan");
    if (batch > 0 && !d_Z) return fail(ZM_EINVAL, "null output pointer");
    zm_status st = run_spectra(p, d_polar, batch, (long long)p->R * p->A, d_ws, ws_bytes, stream, 1);
    if (st == ZM_OK) st = run_project(p, batch, d_Z, d_ws, ws_bytes, stream);
    return noted(st, p, batch, stream, "zm_moments_polar");
}

zm_status zm_resample_polar(zm_plan_t p, const void* d_images, int batch, long long image_stride, void* d_polar,
                            zm_stream_t stream) {
    if (!p) return fail(ZM_EINVAL, "null plan");
    if (batch < 0 || batch > 65535) return fail(ZM_EINVAL, "batch must be in [0, 65535]");
    if (batch == 0) return ZM_OK;
    if (!d_images || !d_polar) return fail(ZM_EINVAL, "null input or output pointer");
    if (batch > 1 && image_stride < (long long)p->H * p->W) return fail(ZM_EINVAL, "image_stride must be >= H * W");
    if (!resample_supported(p->A)) return fail(ZM_EUNSUPPORTED, "the resampler needs angles a power of two in [256, 4096]");
    ZM_DEVICE(p->device);
    hipError_t e = launch_resample(p, d_images, image_stride, batch, d_polar, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "resample kernel launch");
    return noted(ZM_OK, p, batch, stream, "zm_resample_polar");
}

size_t zm_static_scratch_bytes(void) { return kStaticScratchBytes; }

zm_status zm_moments_static(zm_plan_t p, const void* d_images, int batch, long long image_stride, void* d_Z,
                            zm_stream_t stream) {
    if (!p) return fail(ZM_EINVAL, "null plan");
    if (batch < 0) return fail(ZM_EINVAL, "negative batch");
    if (batch == 0) return ZM_OK;
    if (!d_Z) return fail(ZM_EINVAL, "null output pointer");
    if (batch > 1 && image_stride < (long long)p->H * p->W) return fail(ZM_EINVAL, "image_stride must be >= H * W");
    const size_t need = workspace_bytes(p, batch);
    if (need > kStaticScratchBytes) {
        size_t fit = 0;
        while (fit < 65535 && workspace_bytes(p, (int)fit + 1) <= kStaticScratchBytes) ++fit;
        return fail(ZM_EINVAL, "batch needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                                   std::to_string(kStaticScratchBytes) + " bytes (at most " + std::to_string(fit) +
                                   " frames of this plan per call)");
    }
    ZM_DEVICE(p->device);
    void* ws = nullptr;
    zm_status st = scratch_address(p->device, &ws);
    if (st != ZM_OK) return st;
    st = run_spectra(p, d_images, batch, image_stride, ws, kStaticScratchBytes, stream, 0);
    if (st == ZM_OK) st = run_project(p, batch, d_Z, ws, kStaticScratchBytes, stream);
    if (st != ZM_OK) return st;
    log_msg(kLogDebug, "zm_moments_static: plan %p, batch %d, stream %p", (void*)p, batch, stream);
    return note_call(p, (hipStream_t)stream, false);
}

zm_status zm_count_nonfinite(zm_plan_t p, const void* d_Z, int batch, int* d_counts, zm_stream_t stream) {
    if (!p) return fail(ZM_EINVAL, "null plan");
    if (batch < 0 || batch > 65535) return fail(ZM_EINVAL, "batch must be in [0, 65535]");
    if (batch == 0) return ZM_OK;
    if (!d_Z || !d_counts) return fail(ZM_EINVAL, "null moments or counts pointer");
    ZM_DEVICE(p->device);
    hipError_t e = launch_count_nonfinite(p, d_Z, batch, d_counts, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "non-finite count kernel launch");
    log_msg(kLogDebug, "zm_count_nonfinite: plan %p, batch %d, stream %p", (void*)p, batch, stream);
    return ZM_OK;
}

zm_status zm_recon_workspace_size(zm_plan_t p, int batch, size_t* bytes) {
    if (!p || !bytes) return fail(ZM_EINVAL, "null plan or output");
    if (batch < 0) return fail(ZM_EINVAL, "negative batch");
    const size_t nblk = recon_reduce_blocks(p);
    *bytes = align256((size_t)batch * nblk * kErrParts * sizeof(double)) +
             align256((size_t)batch * kErrOut * sizeof(double));
    return ZM_OK;
}

zm_status zm_reconstruct(zm_plan_t p, const void* d_Z, int batch, void* d_out, int kind, int flags,
                         const void* d_ref, void* d_ws, size_t ws_bytes, zm_stream_t stream) {
    if (!p) return fail(ZM_EINVAL, "null plan");
    if (batch < 0 || batch > 65535) return fail(ZM_EINVAL, "batch must be in [0, 65535]");
    if (kind != ZM_RECON_POLAR && kind != ZM_RECON_CARTESIAN) return fail(ZM_EINVAL, "unknown reconstruction kind");
    if (flags & ~(ZM_RECON_ONESIDED | ZM_RECON_MINMAX)) return fail(ZM_EINVAL, "unknown reconstruction flags");
    if ((flags & ZM_RECON_MINMAX) && kind != ZM_RECON_CARTESIAN)
        return fail(ZM_EINVAL, "ZM_RECON_MINMAX applies to Cartesian reconstructions");
    if (batch == 0) return ZM_OK;
    if (!d_Z || !d_out) return fail(ZM_EINVAL, "null device pointer");
    if (flags & ZM_RECON_MINMAX) {
        size_t need = 0;
        zm_recon_workspace_size(p, batch, &need);
        if (!d_ref || !d_ws || ws_bytes < need)
            return fail(ZM_EINVAL, "ZM_RECON_MINMAX needs d_ref and a workspace of zm_recon_workspace_size bytes");
    }
    ZM_DEVICE(p->device);
    hipStream_t s = (hipStream_t)stream;
    const int one = (flags & ZM_RECON_ONESIDED) ? 1 : 0;
    hipError_t e = kind == ZM_RECON_POLAR ? launch_recon_polar(p, d_Z, batch, d_out, one, s)
                                          : launch_recon_cart(p, d_Z, batch, d_out, one, s);
    if (e != hipSuccess) return hip_fail(e, "reconstruction kernel launch");
    if (flags & ZM_RECON_MINMAX) {
        double* part = (double*)d_ws;
        double* mm = (double*)((char*)d_ws + align256((size_t)batch * recon_reduce_blocks(p) * 4 * sizeof(double)));
        e = launch_minmax(p, d_ref, d_out, batch, part, mm, s);
        if (e != hipSuccess) return hip_fail(e, "min-max kernel launch");
    }
    return note_call(p, s);
}

zm_status zm_recon_error(zm_plan_t p, const void* d_ref, const void* d_recon, int batch, double* host_out,
                         void* d_ws, size_t ws_bytes, zm_stream_t stream) {
    if (!p) return fail(ZM_EINVAL, "null plan");
    if (batch < 0 || batch > 65535) return fail(ZM_EINVAL, "batch must be in [0, 65535]");
    if (batch == 0) return ZM_OK;
    size_t need = 0;
    zm_recon_workspace_size(p, batch, &need);
    if (!d_ref || !d_recon || !host_out || !d_ws || ws_bytes < need)
        return fail(ZM_EINVAL, "null pointer or workspace smaller than zm_recon_workspace_size");
    ZM_DEVICE(p->device);
    hipStream_t s = (hipStream_t)stream;
    double* part = (double*)d_ws;
    double* out =
        (double*)((char*)d_ws + align256((size_t)batch * recon_reduce_blocks(p) * kErrParts * sizeof(double)));
    hipError_t e = launch_recon_error(p, d_ref, d_recon, batch, part, out, s);
    if (e != hipSuccess) return hip_fail(e, "error kernel launch");
    ZM_HIP(hipMemcpyAsync(host_out, out, (size_t)batch * kErrOut * sizeof(double), hipMemcpyDeviceToHost, s));
    ZM_HIP(hipStreamSynchronize(s));
    return ZM_OK;
}

static long isqrt_l(long v) {
    long r = (long)std::sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

zm_status zm_pad_size(int n, int* size, int* offset) {
    if (n < 1 || n > 1000000 || !size || !offset) return fail(ZM_EINVAL, "n must be >= 1 and outputs non-null");
    // floor(n (sqrt 2 - 1)) = floor(sqrt(2 n^2)) - n, and floor(x / 2) = floor(floor(x) / 2)
    const long fl = isqrt_l(2L * n * n) - n;
    *size = (int)(n + fl + 20);
    *offset = (int)(fl / 2 + 10);
    return ZM_OK;
}

zm_status zm_embed(const void* d_src, int n, int batch, void* d_dst, int is_double, zm_stream_t stream) {
    int size = 0, off = 0;
    zm_status st = zm_pad_size(n, &size, &off);
    if (st != ZM_OK) return st;
    if (batch < 0 || batch > 65535) return fail(ZM_EINVAL, "batch must be in [0, 65535]");
    if (batch == 0) return ZM_OK;
    if (!d_src || !d_dst) return fail(ZM_EINVAL, "null device pointer");
    hipError_t e = launch_embed(d_src, n, n, (long long)n * n, d_dst, size, off, off, batch, is_double ? 1 : 0,
                                (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "embed kernel launch");
    return ZM_OK;
}

zm_status zm_destroy(zm_plan_t p) {
    if (!p) return fail(ZM_EINVAL, "null plan");
    zm::DeviceGuard guard(p->device);  // frees on the plan's device even if selecting it failed
    {
        std::lock_guard<std::mutex> lk(p->mu);
        if (p->batch_refs > 0) return fail(ZM_EBUSY, "a batch built on this plan still exists; destroy it first");
        for (auto& d : p->done)
            if (hipEventQuery(d.second) == hipErrorNotReady)
                return fail(ZM_EBUSY, "work enqueued on this plan has not completed; synchronise its stream first");
    }
    log_msg(kLogInfo, "plan %p destroyed", (void*)p);
    free_plan(p);
    return ZM_OK;
}

}  // extern "C"
