// One Zernike moment of N x N frames by the Cartesian pixel sum of eq. (6)
// (eq. (14) with the Neumann factor of eq. (15)): every disk pixel centre
// contributes f(x, y) R_nm(rho) exp(-j m theta), no interpolation.
//
// The 8-point symmetry of the square grid (Sec. 2: the symmetry of
// exp(-j m theta), and Fig. 5's timings) groups the pixels into orbits
// (+-X, +-Y), (+-Y, +-X) of one radius.  With w = exp(-j m theta) of the
// first-octant member (X, Y), X >= Y >= 0, the eight angles give
//     G = w P1 + conj(w) P2,
//     P1 = f(X, Y) + (-1)^m f(-X, -Y) + j^m f(Y, -X) + (-j)^m f(-Y, X),
//     P2 = f(X, -Y) + (-1)^m f(-X, Y) + (-j)^m f(Y, X) + j^m f(-Y, -X),
// so R_nm and w are evaluated once per orbit; orbits on a diagonal or an
// axis (and the centre of an odd grid) list their members 2 (8) times and
// are weighted 1/2 (1/8).  rho^m w = ((X - jY) / N)^m by binary powering, and
// R_nm / rho^m = (-1)^k P_k^(m,0)(1 - 2 rho^2), k = (n - m) / 2, by the
// three-term Jacobi recurrence (the polynomial of eq. (2); the coefficients,
// which depend on k and m only, are built in LDS by each workgroup).
//
// Layout: a workgroup owns a 32 x 32 tile of first-octant orbits (quadrant
// indices u >= v) of one frame and stages the tile's eight mirror blocks in
// LDS with row-contiguous loads (all of a thread's loads in flight before the
// first LDS write; the tile grid is shifted so that tile columns start on
// 128-byte lines), so the transposed members (+-Y, +-X) are not gathered
// down columns.  Each thread's 4 orbits share one pass of the recurrence.
// Tiles with no orbit inside the disk (about a fifth of them) skip their
// loads and write a zero partial.  Partial sums per tile, then a fixed-order
// reduction per frame: results do not depend on timing.
#include <hip/hip_runtime.h>

#include <cmath>

#include "zm_internal.h"

namespace {

using zm::fail;
using zm::hip_fail;

constexpr int kT = 32;  // orbit tile side
constexpr int kThreads = 256;
constexpr int kMaxSide = 32768;

// quadrant index u -> doubled coordinate X (units of half a pixel), and the
// column / row of the +X / +Y member
__device__ __forceinline__ long xval(int u, int odd) { return odd ? 2L * u : 2L * u + 1; }
__device__ __forceinline__ int col_p(int u, int N, int odd) { return odd ? (N - 1) / 2 + u : N / 2 + u; }
__device__ __forceinline__ int row_p(int v, int N, int odd) { return odd ? (N - 1) / 2 - v : N / 2 - 1 - v; }

__global__ __launch_bounds__(kThreads) void cart_moment_kernel(const float* __restrict__ img, long long stride, int N,
                                                               int n, int m, int vec, double* __restrict__ part) {
    __shared__ float blk[8][kT][kT + 1];
    __shared__ double red[2][kThreads / 64];
    // (alpha, beta, gamma) of step k, (-1)^k folded in, k = 1..K: 3 (K + 1)
    // doubles of dynamic LDS, so low orders leave room for more workgroups
    extern __shared__ double cf[];
    const int tid = threadIdx.x, b = blockIdx.y;
    const int odd = N & 1, Q = odd ? (N + 1) / 2 : N / 2;
    // tile t -> (tu, tv), tv <= tu, t = tu (tu + 1) / 2 + tv
    const int t = (int)blockIdx.x;
    int tu = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((tu + 1) * (tu + 2) / 2 <= t) ++tu;
    while (tu * (tu + 1) / 2 > t) --tu;
    const int tv = t - tu * (tu + 1) / 2;
    // the tile grid starts sh indices before u = 0 so that tile columns begin
    // on 128-byte lines (the +X column of index u is c0 + u)
    const int c0 = odd ? (N - 1) / 2 : N / 2, sh = c0 % kT;
    const int u0 = tu * kT - sh, v0 = tv * kT - sh;
    // no orbit of the tile inside the disk (its corner nearest the centre is
    // outside): no loads, a zero partial, so the reduction keeps its order
    {
        const long Xn = xval(max(u0, 0), odd), Yn = xval(max(v0, 0), odd);
        if (Xn * Xn + Yn * Yn > (long)N * N) {
            if (tid == 0) {
                double* o = part + ((size_t)b * gridDim.x + t) * 2;
                o[0] = 0.0;
                o[1] = 0.0;
            }
            return;
        }
    }
    const int K = (n - m) / 2;
    for (int k = 1 + tid; k <= K; k += kThreads) {
        const double kk = k, am = m;
        double al, be, ga;
        if (k == 1) {
            al = 0.5 * (am + 2.0);
            be = 0.5 * am;
            ga = 0.0;
        } else {
            const double a1 = 2.0 * kk * (kk + am) * (2.0 * kk + am - 2.0);
            al = (2.0 * kk + am - 1.0) * (2.0 * kk + am) * (2.0 * kk + am - 2.0) / a1;
            be = (2.0 * kk + am - 1.0) * am * am / a1;
            ga = 2.0 * (kk + am - 1.0) * (kk - 1.0) * (2.0 * kk + am) / a1;
        }
        cf[3 * k] = -al;
        cf[3 * k + 1] = -be;
        cf[3 * k + 2] = -ga;
    }
    // blocks 0..3: rows of +-Y (index v), columns of +-X (index u): f(+-X, +-Y) at [v][u]
    // blocks 4..7: rows of +-X (index u), columns of +-Y (index v): f(+-Y, +-X) at [u][v]
    // bit 0 of the block: the row's coordinate negated; bit 1: the column's
    const float* f = img + (size_t)b * (size_t)stride;
    // all of a thread's loads are issued before any is written to LDS
    if (vec) {
        // 16-byte loads (N and the frame stride multiples of 4): with the grid
        // shift, the +X columns of a tile row start at a multiple of 32 and
        // the -X columns end just below one, so a tile row is 8 aligned float4
        // that lie wholly inside or wholly outside the frame; the -X pieces
        // come in descending column order
        constexpr int kPer4 = 8 * kT * (kT / 4) / kThreads;
        float4 v4[kPer4];
#pragma unroll
        for (int i = 0; i < kPer4; ++i) {
            const int e = tid + kThreads * i;
            const int s = e / (kT * kT / 4), a = (e / (kT / 4)) % kT, q = e % (kT / 4);
            const int ri = (s < 4 ? v0 : u0) + a, ci0 = s < 4 ? u0 : v0;
            const int base = (s & 2) ? N - kT - (c0 + ci0) + 4 * q : c0 + ci0 + 4 * q;  // first column of the piece
            v4[i] = float4{0.f, 0.f, 0.f, 0.f};
            if (ri >= 0 && ri < Q && base >= 0 && base + 3 <= N - 1) {
                const int row = (s & 1) ? N - 1 - row_p(ri, N, odd) : row_p(ri, N, odd);
                v4[i] = *reinterpret_cast<const float4*>(f + (size_t)row * N + base);
            }
        }
#pragma unroll
        for (int i = 0; i < kPer4; ++i) {
            const int e = tid + kThreads * i;
            const int s = e / (kT * kT / 4), a = (e / (kT / 4)) % kT, q = e % (kT / 4);
            const int ci0 = s < 4 ? u0 : v0;
            const float w[4] = {v4[i].x, v4[i].y, v4[i].z, v4[i].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = (s & 2) ? kT - 1 - 4 * q - j : 4 * q + j;  // tile column of element j
                blk[s][a][c] = ci0 + c >= 0 ? w[j] : 0.f;  // indices below 0 belong to the other side
            }
        }
    } else {
        constexpr int kPer = 8 * kT * kT / kThreads;
        float vals[kPer];
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = tid + kThreads * i;
            const int s = e / (kT * kT), a = (e / kT) % kT, c = e % kT;
            const int ri = (s < 4 ? v0 : u0) + a, ci = (s < 4 ? u0 : v0) + c;
            vals[i] = 0.f;
            if (ri >= 0 && ci >= 0 && ri < Q && ci < Q) {
                const int row = (s & 1) ? N - 1 - row_p(ri, N, odd) : row_p(ri, N, odd);
                const int col = (s & 2) ? N - 1 - col_p(ci, N, odd) : col_p(ci, N, odd);
                vals[i] = f[(size_t)row * N + col];
            }
        }
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = tid + kThreads * i;
            blk[e / (kT * kT)][(e / kT) % kT][e % kT] = vals[i];
        }
    }
    __syncthreads();

    const double sgn = (m & 1) ? -1.0 : 1.0;
    const double jr = (m & 1) ? 0.0 : ((m & 2) ? -1.0 : 1.0);  // j^m = jr + j ji
    const double ji = (m & 1) ? ((m & 2) ? -1.0 : 1.0) : 0.0;
    const double invN = 1.0 / (double)N;
    // the thread's 4 orbits run through the recurrence together: one read of
    // each coefficient per step and 4 independent FP64 chains; orbits outside
    // the first octant or the disk carry weight 0
    constexpr int kOrb = kT * kT / kThreads;
    double xs[kOrb], gr[kOrb], gi[kOrb], wgt[kOrb];
#pragma unroll
    for (int e = 0; e < kOrb; ++e) {
        const int ul = tid % kT, vl = tid / kT + (kThreads / kT) * e;
        const int u = u0 + ul, v = v0 + vl;
        const long X = xval(u, odd), Y = xval(v, odd), P = X * X + Y * Y;
        const bool in = v >= 0 && u < Q && v <= u && P <= (long)N * N;
        const double fXY = blk[0][vl][ul], fXmY = blk[1][vl][ul], fmXY = blk[2][vl][ul], fmXmY = blk[3][vl][ul];
        const double fYX = blk[4][ul][vl], fYmX = blk[5][ul][vl], fmYX = blk[6][ul][vl], fmYmX = blk[7][ul][vl];
        // j^m a + (-j)^m c = jr (a + c) + j ji (a - c)
        const double p1r = fXY + sgn * fmXmY + jr * (fYmX + fmYX), p1i = ji * (fYmX - fmYX);
        const double p2r = fXmY + sgn * fmXY + jr * (fYX + fmYmX), p2i = ji * (fmYmX - fYX);
        // z^m = rho^m w, z = (X - jY) / N
        double zr = (double)X * invN, zi = -(double)Y * invN, wr = 1.0, wi = 0.0;
        for (int ee = m; ee; ee >>= 1) {
            if (ee & 1) {
                const double tr = wr * zr - wi * zi;
                wi = wr * zi + wi * zr;
                wr = tr;
            }
            const double sr = zr * zr - zi * zi;
            zi = 2.0 * zr * zi;
            zr = sr;
        }
        // G = z^m P1 + conj(z^m) P2
        // orbits outside the disk run the recurrence at x = 0 (bounded) with G = 0
        gr[e] = in ? wr * (p1r + p2r) + wi * (p2i - p1i) : 0.0;
        gi[e] = in ? wr * (p1i + p2i) + wi * (p1r - p2r) : 0.0;
        xs[e] = in ? 1.0 - 2.0 * (double)P * invN * invN : 0.0;
        wgt[e] = !in ? 0.0 : (X == 0 ? 0.125 : ((X == Y || Y == 0) ? 0.5 : 1.0));
    }
    double q1[kOrb], q2[kOrb];
#pragma unroll
    for (int e = 0; e < kOrb; ++e) {
        q1[e] = 1.0;
        q2[e] = 0.0;
    }
    for (int k = 1; k <= K; ++k) {
        const double al = cf[3 * k], be = cf[3 * k + 1], ga = cf[3 * k + 2];
#pragma unroll
        for (int e = 0; e < kOrb; ++e) {
            const double q = (al * xs[e] + be) * q1[e] + ga * q2[e];
            q2[e] = q1[e];
            q1[e] = q;
        }
    }
    double accr = 0.0, acci = 0.0;
#pragma unroll
    for (int e = 0; e < kOrb; ++e) {
        accr += wgt[e] * q1[e] * gr[e];
        acci += wgt[e] * q1[e] * gi[e];
    }
    // fixed-order reduction: a butterfly within each wave, then the waves in order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        accr += __shfl_xor(accr, o, 64);
        acci += __shfl_xor(acci, o, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = accr;
        red[1][tid >> 6] = acci;
    }
    __syncthreads();
    if (tid == 0) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            sr += red[0][w];
            si += red[1][w];
        }
        double* o = part + ((size_t)b * gridDim.x + t) * 2;
        o[0] = sr;
        o[1] = si;
    }
}

// out[b] = scale * sum over tiles (fixed order), conjugated for m < 0
__global__ __launch_bounds__(kThreads) void cart_final_kernel(const double* __restrict__ part, int ntiles,
                                                              double scale, int conj, double* __restrict__ out) {
    __shared__ double red[2][kThreads];
    const int b = blockIdx.x, tid = threadIdx.x;
    double sr = 0.0, si = 0.0;
    for (int k = tid; k < ntiles; k += kThreads) {
        sr += part[((size_t)b * ntiles + k) * 2];
        si += part[((size_t)b * ntiles + k) * 2 + 1];
    }
    red[0][tid] = sr;
    red[1][tid] = si;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] += red[0][tid + s];
            red[1][tid] += red[1][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[2 * (size_t)b] = scale * red[0][0];
        out[2 * (size_t)b + 1] = (conj ? -scale : scale) * red[1][0];
    }
}

int tiles_of(int N) {
    const int Q = (N & 1) ? (N + 1) / 2 : N / 2;
    const int sh = ((N & 1) ? (N - 1) / 2 : N / 2) % kT;  // grid shift of the kernel
    const int T = (Q + sh + kT - 1) / kT;
    return T * (T + 1) / 2;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

zm_status zm_cartesian_workspace_size(int n_side, int batch, size_t* bytes) {
    if (!bytes || n_side < 1 || n_side > kMaxSide || batch < 0)
        return fail(ZM_EINVAL, "n_side must be in [1, 32768], batch >= 0 and bytes non-null");
    *bytes = align256((size_t)batch * tiles_of(n_side) * 2 * sizeof(double));
    return ZM_OK;
}

zm_status zm_moment_cartesian(const void* d_frames, int n_side, int batch, long long frame_stride, int n, int m,
                              int neumann, double* d_out, void* d_ws, size_t ws_bytes, zm_stream_t stream) {
    const int am = m < 0 ? -m : m;
    if (n < 0 || n > zm::kMaxTableOrder || am > n || ((n - am) & 1))
        return fail(ZM_EINVAL, "need 0 <= n <= 500, |m| <= n and n - |m| even");
    if (n_side < 1 || n_side > kMaxSide) return fail(ZM_EINVAL, "n_side must be in [1, 32768]");
    if (batch < 0 || batch > 65535) return fail(ZM_EINVAL, "batch must be in [0, 65535]");
    if (batch == 0) return ZM_OK;
    if (frame_stride < (long long)n_side * n_side) return fail(ZM_EINVAL, "frame_stride smaller than n_side^2");
    size_t need = 0;
    zm_cartesian_workspace_size(n_side, batch, &need);
    if (!d_frames || !d_out || !d_ws || ws_bytes < need)
        return fail(ZM_EINVAL, "null pointer or workspace smaller than zm_cartesian_workspace_size");
    hipStream_t s = (hipStream_t)stream;
    const int ntiles = tiles_of(n_side);
    // 16-byte loads when every frame row starts 16-byte aligned
    const int vec = (n_side % 4 == 0 && frame_stride % 4 == 0 && ((uintptr_t)d_frames & 15) == 0) ? 1 : 0;
    const size_t cf_bytes = 3 * (size_t)((n - am) / 2 + 1) * sizeof(double);
    hipLaunchKernelGGL(cart_moment_kernel, dim3(ntiles, batch), dim3(kThreads), cf_bytes, s,
                       (const float*)d_frames, frame_stride, n_side, n, am, vec, (double*)d_ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "Cartesian moment kernel launch");
    const double eps = (neumann && am == 0) ? 2.0 : 1.0;
    const double delta = 2.0 / n_side;
    const double scale = (double)(n + 1) / (M_PI * eps) * delta * delta;
    hipLaunchKernelGGL(cart_final_kernel, dim3(batch), dim3(kThreads), 0, s, (const double*)d_ws, ntiles, scale,
                       m < 0 ? 1 : 0, d_out);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "Cartesian reduction launch");
    return ZM_OK;
}

}  // extern "C"
