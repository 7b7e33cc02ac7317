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
template <typename ZT, typename OT>
__global__ __launch_bounds__(kThreads) void recon_cart_kernel(const ZT* __restrict__ Zall, int Mtot, int nmax, int H,
                                                              int W, const double* __restrict__ jac, int neumann,
                                                              int one_sided, OT* __restrict__ out) {
    const int b = blockIdx.y;
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= (long)H * W) return;
    const int i = (int)(p / W), jx = (int)(p % W);
    const int D = min(H, W);
    const long X = 2L * jx - (W - 1), Y = (long)(H - 1) - 2L * i;
    const long P = X * X + Y * Y;
    OT* o = out + (size_t)b * H * W;
    if (P > (long)D * D) {
        o[p] = (OT)0;
        return;
    }
    const ZT* Z = Zall + (size_t)b * Mtot * 2;
    const double rho2 = (double)P / ((double)D * (double)D);
    const double rho = sqrt(rho2);
    const double x = 1.0 - 2.0 * rho2;
    const double th = atan2((double)Y, (double)X);
    const double c1 = cos(th), s1 = sin(th);
    double cm = 1.0, sm = 0.0;  // cos, sin of m theta (complex powers of exp(i theta))
    double rm = 1.0;            // rho^m
    double acc = 0.0;
    for (int m = 0; m <= nmax; ++m) {
        int idx = zm::canon_index(m, m);
        double sr = zre(Z, idx), si = zim(Z, idx);  // Q_0 = 1
        double q1 = 1.0, q2 = 0.0;                    // Q_{k-1}, Q_{k-2}
#pragma unroll 4
        for (int n = m + 2; n <= nmax; n += 2) {
            idx = zm::canon_index(n, m);
            const double* J = jac + 3 * (size_t)idx;
            const double q = (J[0] * x + J[1]) * q1 + J[2] * q2;
            q2 = q1;
            q1 = q;
            sr += q * zre(Z, idx);
            si += q * zim(Z, idx);
        }
        acc += coef_m(m, neumann, one_sided) * rm * (sr * cm - si * sm);
        const double cn = cm * c1 - sm * s1, sn = sm * c1 + cm * s1;
        cm = cn;
        sm = sn;
        rm *= rho;
    }
    o[p] = (OT)acc;
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
    const long npx = (long)p->H * p->W;
    dim3 grid((unsigned)((npx + kThreads - 1) / kThreads), batch);
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
