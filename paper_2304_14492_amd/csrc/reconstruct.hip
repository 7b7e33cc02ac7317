// Image reconstruction from moments (Sec. 2.2, eq. (9)), the reconstruction
// error of eq. (13) (Sec. 2.4) and the per-band min-max renormalisation
// (Sec. 2.3, Sec. 3).  All accumulation is FP64.
//
// eq. (9): f~(rho, theta) = Re sum_n sum_{m=-n..n, n-m even} Z_nm R_nm(rho) exp(j m theta).
// Only m >= 0 is stored; with Z_{n,-m} = conj(Z_nm) (Sec. 2) every m > 0
// term appears twice, so f~ = sum_{n,m>=0} c_m Re(Z_nm exp(j m theta)) R_nm(rho)
// with c_0 = eps_0 (Neumann factor multiplied back when the plan divided by
// it, eq. (14)-(15)) and c_m = 2 otherwise.  The one-sided variant sums
// Re(Z_nm exp(j m theta)) R_nm over the stored moments once (c_m = 1).
//
// Polar nodes use the plan's FP64 table of eq. (7).  Pixel centres need R_nm
// at arbitrary rho; there it is evaluated as
//     R_n^m(rho) = (-1)^k rho^m P_k^(m,0)(1 - 2 rho^2),  k = (n - m)/2,
// with the three-term recurrence of the Jacobi polynomials (forward-stable on
// [-1, 1]) -- the same polynomial as eq. (2).
#include <hip/hip_runtime.h>

#include "zm_internal.h"

namespace {

constexpr int kThreads = 256;

template <typename ZT>
__device__ __forceinline__ double zre(const ZT* Z, size_t i) { return (double)Z[2 * i]; }
template <typename ZT>
__device__ __forceinline__ double zim(const ZT* Z, size_t i) { return (double)Z[2 * i + 1]; }

__device__ __forceinline__ double coef_m(int m, int neumann, int one_sided) {
    if (one_sided) return 1.0;
    if (m == 0) return neumann ? 2.0 : 1.0;
    return 2.0;
}

// One workgroup per (frame, ring): G[m] = sum_n Z_nm R_nm(rho_r) in LDS, then
// f~[r][a] = sum_m c_m Re(G[m] exp(2 pi i m a / A)).
template <typename ZT, typename OT>
__global__ __launch_bounds__(kThreads) void recon_polar_kernel(const ZT* __restrict__ Zall, int Mtot, int nmax,
                                                               int R, int A, const double* __restrict__ table,
                                                               const double* __restrict__ trig, int neumann,
                                                               int one_sided, OT* __restrict__ out) {
    const int r = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const ZT* Z = Zall + (size_t)b * Mtot * 2;
    __shared__ double gre[zm::kMaxTableOrder + 1], gim[zm::kMaxTableOrder + 1];
    for (int m = tid; m <= nmax; m += kThreads) {
        double sr = 0.0, si = 0.0;
        for (int n = m; n <= nmax; n += 2) {
            const int idx = zm::canon_index(n, m);
            const double t = table[(size_t)idx * R + r];
            sr += t * zre(Z, idx);
            si += t * zim(Z, idx);
        }
        const double c = coef_m(m, neumann, one_sided);
        gre[m] = c * sr;
        gim[m] = c * si;
    }
    __syncthreads();
    for (int a = tid; a < A; a += kThreads) {
        double acc = 0.0;
        long j = 0;  // (m * a) mod A
        for (int m = 0; m <= nmax; ++m) {
            // Re(G (cos + i sin)) = Gr cos - Gi sin, cos/sin of 2 pi m a / A
            acc += gre[m] * trig[2 * j] - gim[m] * trig[2 * j + 1];
            j += a;
            if (j >= A) j -= A * (j / A);
        }
        out[((size_t)b * R + r) * A + a] = (OT)acc;
    }
}

// One thread per pixel centre: rho^2 = P / D^2 with the integer
// P = (2j - (W-1))^2 + ((H-1) - 2i)^2; pixels with rho > 1 are set to 0.
// Per m, S_m = sum_k Z_{m+2k,m} Q_k(x) with the plan's recurrence
// coefficients (jac: alpha, beta, gamma per moment; the same for every pixel,
// read with scalar loads), then f~ += c_m rho^m Re(S_m exp(j m theta)).
// pixels per thread of the pixel-centre kernel: they share every read of the
// staged coefficients, which would otherwise outrun the FP64 pipes.  A
// workgroup covers 64 x 16 pixels, each wave a 16 x 16 tile (compact, so
// waves wholly outside the disk skip the recurrence), each thread one column
// of 4 pixels 4 rows apart.
constexpr int kPix = 4;
constexpr int kTileW = 64, kTileH = 16;

template <typename ZT, typename OT>
__global__ __launch_bounds__(kThreads) void recon_cart_kernel(const ZT* __restrict__ Zall, int Mtot, int nmax, int H,
                                                              int W, const double* __restrict__ jac, int neumann,
                                                              int one_sided, OT* __restrict__ out) {
    // Column m of the recurrence, staged in LDS for the whole workgroup:
    // entry e (n = m + 2e) holds (J0, J1, J2) of step e (e >= 1) and
    // (Re, Im) Z_nm as doubles.  Two buffers: column m + 1 is loaded into
    // registers while column m is used, so the loads' latency is hidden.
    static_assert(zm::kMaxTableOrder / 2 + 1 <= kThreads, "one column entry per thread");
    __shared__ double col[2][zm::kMaxTableOrder / 2 + 1][6];
    const int b = blockIdx.z, tid = threadIdx.x;
    const long npx = (long)H * W;
    const int col0 = blockIdx.x * kTileW + (tid >> 6) * 16 + (tid & 15);
    const int row0 = blockIdx.y * kTileH + ((tid & 63) >> 4);
    const int D = min(H, W);
    const ZT* Z = Zall + (size_t)b * Mtot * 2;
    // thread's pixels: (row0 + 4k, col0); pixels outside the disk run the
    // recurrence at x = 0 (bounded) and write 0
    double x[kPix], rho[kPix], c1[kPix], s1[kPix], cm[kPix], sm[kPix], rm[kPix], acc[kPix];
    bool in[kPix];
    bool any = false;
#pragma unroll
    for (int k = 0; k < kPix; ++k) {
        const int i = row0 + 4 * k, jx = col0;
        const bool live = i < H && jx < W;
        const long X = 2L * jx - (W - 1), Y = (long)(H - 1) - 2L * i;
        const long P = X * X + Y * Y;
        in[k] = live && P <= (long)D * D;
        any = any || in[k];
        const double rho2 = in[k] ? (double)P / ((double)D * (double)D) : 0.5;
        rho[k] = in[k] ? sqrt(rho2) : 0.0;
        x[k] = 1.0 - 2.0 * rho2;
        const double th = in[k] ? atan2((double)Y, (double)X) : 0.0;
        c1[k] = cos(th);
        s1[k] = sin(th);
        cm[k] = 1.0;  // cos, sin of m theta (complex powers of exp(i theta))
        sm[k] = 0.0;
        rm[k] = 1.0;  // rho^m
        acc[k] = 0.0;
    }
    // entry e = tid of column m (nmax - m >= 2 e), loaded into registers
    double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0, r4 = 0.0;
    auto fetch = [&](int m) {
        if (2 * tid <= nmax - m) {
            const int idx = zm::canon_index(m + 2 * tid, m);
            if (tid > 0) {
                r0 = jac[3 * (size_t)idx];
                r1 = jac[3 * (size_t)idx + 1];
                r2 = jac[3 * (size_t)idx + 2];
            }
            r3 = zre(Z, idx);
            r4 = zim(Z, idx);
        }
    };
    auto stage = [&](int m, int buf) {
        if (2 * tid <= nmax - m) {
            double* c = col[buf][tid];
            c[0] = r0;
            c[1] = r1;
            c[2] = r2;
            c[3] = r3;
            c[4] = r4;
        }
    };
    fetch(0);
    stage(0, 0);
    __syncthreads();
    for (int m = 0; m <= nmax; ++m) {
        const int cur = m & 1;
        if (m < nmax) fetch(m + 1);
        if (any) {
            const double(*cc)[6] = col[cur];
            double sr[kPix], si[kPix], q1[kPix], q2[kPix];
#pragma unroll
            for (int k = 0; k < kPix; ++k) {
                sr[k] = cc[0][3];  // Q_0 = 1
                si[k] = cc[0][4];
                q1[k] = 1.0;  // Q_{k-1}
                q2[k] = 0.0;  // Q_{k-2}
            }
            const int Km = (nmax - m) / 2;
#pragma unroll 2
            for (int e = 1; e <= Km; ++e) {
                const double j0 = cc[e][0], j1 = cc[e][1], j2 = cc[e][2], zr = cc[e][3], zi = cc[e][4];
#pragma unroll
                for (int k = 0; k < kPix; ++k) {
                    const double q = (j0 * x[k] + j1) * q1[k] + j2 * q2[k];
                    q2[k] = q1[k];
                    q1[k] = q;
                    sr[k] += q * zr;
                    si[k] += q * zi;
                }
            }
            const double cf = coef_m(m, neumann, one_sided);
#pragma unroll
            for (int k = 0; k < kPix; ++k) {
                acc[k] += cf * rm[k] * (sr[k] * cm[k] - si[k] * sm[k]);
                const double cn = cm[k] * c1[k] - sm[k] * s1[k], sn = sm[k] * c1[k] + cm[k] * s1[k];
                cm[k] = cn;
                sm[k] = sn;
                rm[k] *= rho[k];
            }
        }
        // buffer cur ^ 1 was last read for column m - 1, before the previous barrier
        if (m < nmax) stage(m + 1, cur ^ 1);
        __syncthreads();
    }
    OT* o = out + (size_t)b * npx;
#pragma unroll
    for (int k = 0; k < kPix; ++k) {
        const int i = row0 + 4 * k;
        if (i < H && col0 < W) o[(long)i * W + col0] = in[k] ? (OT)acc[k] : (OT)0;
    }
}

// eq. (13) per frame over the disk: partial sums per block, then a
// fixed-order reduction (deterministic).  part[b][blk] = {sse, sum f^2, f_max, count}.
template <typename FT, typename RT>
__global__ __launch_bounds__(kThreads) void error_partial_kernel(const FT* __restrict__ f, const RT* __restrict__ g,
                                                                 int H, int W, double* __restrict__ part) {
    const int b = blockIdx.y;
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    __shared__ double sh[zm::kErrParts][kThreads];
    // per pixel of the disk: (f - f~)^2, f^2, |f|, 1, (f - f~)^2 / f^2 where
    // f != 0 (eq. (12) is singular where f = 0), and 1 where f = 0
    double v[zm::kErrParts] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (p < (long)H * W) {
        const int i = (int)(p / W), jx = (int)(p % W);
        const int D = min(H, W);
        const long X = 2L * jx - (W - 1), Y = (long)(H - 1) - 2L * i;
        if (X * X + Y * Y <= (long)D * D) {
            const double fv = (double)f[(size_t)b * H * W + p], gv = (double)g[(size_t)b * H * W + p];
            const double d2 = (fv - gv) * (fv - gv);
            v[0] = d2;
            v[1] = fv * fv;
            v[2] = fabs(fv);
            v[3] = 1.0;
            if (fv != 0.0)
                v[4] = d2 / (fv * fv);
            else
                v[5] = 1.0;
        }
    }
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < zm::kErrParts; ++k) sh[k][t] = v[k];
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int k = 0; k < zm::kErrParts; ++k)
                sh[k][t] = k == 2 ? fmax(sh[k][t], sh[k][t + s]) : sh[k][t] + sh[k][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        double* o = part + ((size_t)b * gridDim.x + blockIdx.x) * zm::kErrParts;
#pragma unroll
        for (int k = 0; k < zm::kErrParts; ++k) o[k] = sh[k][0];
    }
}

__global__ void error_final_kernel(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    double q[zm::kErrParts] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nblk; ++k) {
        const double* r = part + ((size_t)b * nblk + k) * zm::kErrParts;
        for (int c = 0; c < zm::kErrParts; ++c) q[c] = c == 2 ? fmax(q[c], r[c]) : q[c] + r[c];
    }
    const double sse = q[0], sf2 = q[1], fm = q[2], cnt = q[3];
    double* o = out + (size_t)b * zm::kErrOut;
    o[0] = (fm > 0.0 && cnt > 0.0) ? sse / (fm * fm * cnt) : 0.0;  // eq. (13)
    o[1] = sf2 > 0.0 ? sse / sf2 : 0.0;                             // eq. (10)
    o[2] = sse;
    o[3] = fm;
    o[4] = cnt;
    o[5] = q[4];  // eq. (12) over the pixels with f != 0
    o[6] = q[5];  // pixels of the disk with f = 0 (left out of eq. (12))
}

// min / max over the disk of the reference (band) and of the reconstruction.
template <typename FT, typename RT>
__global__ __launch_bounds__(kThreads) void minmax_partial_kernel(const FT* __restrict__ f, const RT* __restrict__ g,
                                                                  int H, int W, double* __restrict__ part) {
    const int b = blockIdx.y;
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    __shared__ double s[4][kThreads];
    const double inf = __builtin_huge_val();
    double flo = inf, fhi = -inf, glo = inf, ghi = -inf;
    if (p < (long)H * W) {
        const int i = (int)(p / W), jx = (int)(p % W);
        const int D = min(H, W);
        const long X = 2L * jx - (W - 1), Y = (long)(H - 1) - 2L * i;
        if (X * X + Y * Y <= (long)D * D) {
            const double fv = (double)f[(size_t)b * H * W + p], gv = (double)g[(size_t)b * H * W + p];
            flo = fhi = fv;
            glo = ghi = gv;
        }
    }
    const int t = threadIdx.x;
    s[0][t] = flo; s[1][t] = fhi; s[2][t] = glo; s[3][t] = ghi;
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if (t < st) {
            s[0][t] = fmin(s[0][t], s[0][t + st]);
            s[1][t] = fmax(s[1][t], s[1][t + st]);
            s[2][t] = fmin(s[2][t], s[2][t + st]);
            s[3][t] = fmax(s[3][t], s[3][t + st]);
        }
        __syncthreads();
    }
    if (t == 0) {
        double* o = part + ((size_t)b * gridDim.x + blockIdx.x) * 4;
        o[0] = s[0][0]; o[1] = s[1][0]; o[2] = s[2][0]; o[3] = s[3][0];
    }
}

__global__ void minmax_final_kernel(const double* __restrict__ part, int nblk, double* __restrict__ mm) {
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    const double inf = __builtin_huge_val();
    double a0 = inf, a1 = -inf, a2 = inf, a3 = -inf;
    for (int k = 0; k < nblk; ++k) {
        const double* q = part + ((size_t)b * nblk + k) * 4;
        a0 = fmin(a0, q[0]); a1 = fmax(a1, q[1]); a2 = fmin(a2, q[2]); a3 = fmax(a3, q[3]);
    }
    double* o = mm + (size_t)b * 4;
    o[0] = a0; o[1] = a1; o[2] = a2; o[3] = a3;
}

// g <- (g - min g) / (max g - min g) * (max f - min f) + min f inside the disk.
template <typename RT>
__global__ __launch_bounds__(kThreads) void minmax_apply_kernel(RT* __restrict__ g, int H, int W,
                                                                const double* __restrict__ mm) {
    const int b = blockIdx.y;
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= (long)H * W) return;
    const int i = (int)(p / W), jx = (int)(p % W);
    const int D = min(H, W);
    const long X = 2L * jx - (W - 1), Y = (long)(H - 1) - 2L * i;
    if (X * X + Y * Y > (long)D * D) return;
    const double* q = mm + (size_t)b * 4;
    const double span = q[3] - q[2];
    const double sc = span > 0.0 ? (q[1] - q[0]) / span : 0.0;
    RT* o = g + (size_t)b * H * W + p;
    *o = (RT)(((double)*o - q[2]) * sc + q[0]);
}

// Embed an n_rows x n_cols image at (off_r, off_c) of a zero size x size grid
// (the preprocessing of Sec. 3 that puts the whole image inside the disk).
template <typename T>
__global__ __launch_bounds__(kThreads) void embed_kernel(const T* __restrict__ src, int n_rows, int n_cols,
                                                         long long src_stride, T* __restrict__ dst, int size,
                                                         int off_r, int off_c) {
    const int b = blockIdx.y;
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= (long)size * size) return;
    const int i = (int)(p / size) - off_r, j = (int)(p % size) - off_c;
    T v = (T)0;
    if (i >= 0 && j >= 0 && i < n_rows && j < n_cols) v = src[(size_t)b * src_stride + (size_t)i * n_cols + j];
    dst[(size_t)b * size * size + p] = v;
}

}  // namespace

namespace zm {

hipError_t launch_embed(const void* src, int n_rows, int n_cols, long long src_stride, void* dst, int size, int off_r,
                        int off_c, int batch, int is_double, hipStream_t s) {
    dim3 grid((unsigned)(((long)size * size + kThreads - 1) / kThreads), batch);
    if (is_double)
        hipLaunchKernelGGL((embed_kernel<double>), grid, dim3(kThreads), 0, s, (const double*)src, n_rows, n_cols,
                           src_stride, (double*)dst, size, off_r, off_c);
    else
        hipLaunchKernelGGL((embed_kernel<float>), grid, dim3(kThreads), 0, s, (const float*)src, n_rows, n_cols,
                           src_stride, (float*)dst, size, off_r, off_c);
    return hipGetLastError();
}

hipError_t launch_recon_polar(const zm_plan_s* p, const void* Z, int batch, void* out, int one_sided, hipStream_t s) {
    dim3 grid(p->R, batch);
    if (p->dtype == ZM_F64)
        hipLaunchKernelGGL((recon_polar_kernel<double, double>), grid, dim3(kThreads), 0, s, (const double*)Z,
                           p->num_moments, p->n_max, p->R, p->A, p->d_table, p->d_trig, p->neumann, one_sided,
                           (double*)out);
    else
        hipLaunchKernelGGL((recon_polar_kernel<float, float>), grid, dim3(kThreads), 0, s, (const float*)Z,
                           p->num_moments, p->n_max, p->R, p->A, p->d_table, p->d_trig, p->neumann, one_sided,
                           (float*)out);
    return hipGetLastError();
}

hipError_t launch_recon_cart(const zm_plan_s* p, const void* Z, int batch, void* out, int one_sided, hipStream_t s) {
    static_assert(kThreads == 4 * 64 && kTileW == 4 * 16 && kTileH == 4 * kPix, "4 waves of 16 x 16 pixels");
    dim3 grid((unsigned)((p->W + kTileW - 1) / kTileW), (unsigned)((p->H + kTileH - 1) / kTileH), batch);
    if (p->dtype == ZM_F64)
        hipLaunchKernelGGL((recon_cart_kernel<double, double>), grid, dim3(kThreads), 0, s, (const double*)Z,
                           p->num_moments, p->n_max, p->H, p->W, p->d_jac, p->neumann, one_sided, (double*)out);
    else
        hipLaunchKernelGGL((recon_cart_kernel<float, float>), grid, dim3(kThreads), 0, s, (const float*)Z,
                           p->num_moments, p->n_max, p->H, p->W, p->d_jac, p->neumann, one_sided, (float*)out);
    return hipGetLastError();
}

size_t recon_reduce_blocks(const zm_plan_s* p) { return ((size_t)p->H * p->W + kThreads - 1) / kThreads; }

hipError_t launch_recon_error(const zm_plan_s* p, const void* f, const void* g, int batch, double* part,
                              double* out, hipStream_t s) {
    const int nblk = (int)recon_reduce_blocks(p);
    dim3 grid(nblk, batch);
    if (p->dtype == ZM_F64)
        hipLaunchKernelGGL((error_partial_kernel<double, double>), grid, dim3(kThreads), 0, s, (const double*)f,
                           (const double*)g, p->H, p->W, part);
    else
        hipLaunchKernelGGL((error_partial_kernel<float, float>), grid, dim3(kThreads), 0, s, (const float*)f,
                           (const float*)g, p->H, p->W, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(error_final_kernel, dim3(batch), dim3(64), 0, s, part, nblk, out);
    return hipGetLastError();
}

hipError_t launch_minmax(const zm_plan_s* p, const void* f, void* g, int batch, double* part, double* mm,
                         hipStream_t s) {
    const int nblk = (int)recon_reduce_blocks(p);
    dim3 grid(nblk, batch);
    if (p->dtype == ZM_F64)
        hipLaunchKernelGGL((minmax_partial_kernel<double, double>), grid, dim3(kThreads), 0, s, (const double*)f,
                           (const double*)g, p->H, p->W, part);
    else
        hipLaunchKernelGGL((minmax_partial_kernel<float, float>), grid, dim3(kThreads), 0, s, (const float*)f,
                           (const float*)g, p->H, p->W, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(minmax_final_kernel, dim3(batch), dim3(64), 0, s, part, nblk, mm);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (p->dtype == ZM_F64)
        hipLaunchKernelGGL((minmax_apply_kernel<double>), grid, dim3(kThreads), 0, s, (double*)g, p->H, p->W, mm);
    else
        hipLaunchKernelGGL((minmax_apply_kernel<float>), grid, dim3(kThreads), 0, s, (float*)g, p->H, p->W, mm);
    return hipGetLastError();
}

}  // namespace zm
