// Pixel -> polar resampling on its own (Sec. 2.5): the bilinear samples
// f^(rho_r, theta_a) of the polar grid of eq. (1), written as a polar image
// P[b][r][a] (R x A per frame) that the angular transform then reads in
// coalesced rows (the from-polar form of the resample + FFT kernel).
//
// Why a kernel of its own: the fused kernel gathers one round of 4 rings per
// workgroup, and a 128-byte row line that the rings cross where they run
// vertically spans 32 rings, so each such line is fetched into L1 by about 8
// rounds on different CUs.  Here a workgroup owns a tile of 32 rings x 64
// base angles (all four quarter turns), so the lines of a band are fetched
// about once per tile.
//
// Sample positions and values are computed exactly as in the fused gather
// (the same base-angle (cos, sin) rotation, sample_pos and bilinear
// expression), so the polar image holds the same bits as the fused kernel's
// gathered samples, and resample + from-polar transform give the same
// spectra as the fused kernel.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_body.h"

namespace {

using namespace zmk;

constexpr int kRB = 32;                 // rings per tile
constexpr int kAB = 64;                 // first-quadrant base angles per tile
constexpr int kThreads = 256;           // 4 waves, 16 base angles each
constexpr int kBW = kAB / (kThreads / 64);
constexpr int kRow = kAB + 2;           // LDS row stride of the output tile
static_assert(kBW == 16 && kRB == 32, "lane maps below assume 16 base angles x 32 rings per wave");

template <typename Real>
struct ResampleArgs {
    const Real* src;
    long long src_stride;  // elements between frames
    int H, W, R, A;
    double cx, cy, safe_s;
    const double* spx;   // ring radius in pixels, R
    const double* trig;  // (cos, sin)(2 pi a / A), FP64
    Real* P;             // polar images, [b][R][A]
};

// One tile: rings [rb, rb + 32) x base angles [b0, b0 + 64) of frame img,
// every quarter turn u of each base angle b (angle b + u A / 4).  A wave
// instruction covers either 32 consecutive rings at 2 base angles ("V": each
// group of 4 lanes holds 4 consecutive rings at one angle) or 4 rings at 16
// consecutive base angles ("H": 4 consecutive angles of one ring per group);
// at angle phi from the x axis a V group spans rows in proportion to
// dr sin(phi), an H group to ds cos(phi) (dr the ring step, ds = 2 pi r / A),
// so V serves the turns whose angle has tan(phi) < ds / dr.  Turns 0, 2 sit
// at the base angle phi, turns 1, 3 at its complement.
template <typename Real>
__device__ __forceinline__ void resample_tile(const ResampleArgs<Real>& g, int img, int rb, int b0, Real* tile) {
    const int H = g.H, W = g.W, R = g.R, A = g.A;
    const double cx = g.cx, cy = g.cy;
    const double* __restrict__ spx = g.spx;
    const double* __restrict__ trig = g.trig;
    const Real* __restrict__ frame = g.src + (size_t)img * (size_t)g.src_stride;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

    const int last = min(rb + kRB, R) - 1;
    const bool check = spx[last] >= g.safe_s;
    // which map each pair of turns uses, from the tile's middle angle and first ring
    bool p_v = true, q_v = false;
    if (R > 1) {
        const int rn = rb + 1 < R ? rb + 1 : rb - 1;
        const double dr = fabs(spx[rn] - spx[rb]);
        const double ratio = 6.283185307179586 * spx[rb] / ((double)A * dr);
        const double phi = 6.283185307179586 * (b0 + 0.5 * kAB) / A;
        const double t = tan(phi);
        p_v = t < ratio;
        q_v = 1.0 / t < ratio;
    }
    // (cos, sin) of this lane's H base angle b0 + 16 w + lane % 16: the table
    // pair of b mod (A / 32) rotated by the pair of (A / 32) floor(b / (A / 32))
    const int kStep = A / 32;
    const int bh = b0 + kBW * w + (lane & 15);
    double ch, sh;
    rotate_pair(trig[2 * (bh % kStep)], trig[2 * (bh % kStep) + 1], trig[2 * kStep * (bh / kStep)],
                trig[2 * kStep * (bh / kStep) + 1], ch, sh);
    // radius of this lane's V ring rb + lane % 32
    const int rv = rb + (lane & 31);
    const double sr_v = rv < R ? spx[rv] : 0.0;

    // per iteration p: V ring rb + lane % 32 at base angle b0 + 16 w + 2 p +
    // lane / 32 (its (cos, sin) held by lane 2 p + lane / 32); H ring
    // rb + 4 p + lane / 16 (its radius held by lane 4 p + lane / 16) at this
    // lane's base angle
    double cvs[8], svs[8], srh[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int src_v = 2 * p + (lane >> 5);
        cvs[p] = __shfl(ch, src_v, 64);
        svs[p] = __shfl(sh, src_v, 64);
        srh[p] = __shfl(sr_v, 4 * p + (lane >> 4), 64);
    }
    // one quarter turn at a time, so that consecutive loads of a wave fall on
    // neighbouring rows and the L1 keeps the lines they share; the 16 loads of
    // a turn are issued before any of its values is stored (rings past R
    // sample at radius 0, inside the frame, and are dropped)
    auto turns = [&](auto checked) {
        constexpr bool CHECK = decltype(checked)::value;
#pragma unroll 1
        for (int u = 0; u < 4; ++u) {
            const bool use_v = (u & 1) ? q_v : p_v;
            Real val[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const double sr = use_v ? sr_v : srh[p];
                const double c = use_v ? cvs[p] : ch, s = use_v ? svs[p] : sh;
                const TapPos<Real> tp = sample_pos<Real>(cx, cy, W, H, sr, c, s, u);
                val[p] = bilinear_idx<Real, CHECK>(frame, H, W, tp.x.i, tp.y.i, tp.x.f, tp.y.f);
            }
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const int rl = use_v ? (lane & 31) : 4 * p + (lane >> 4);
                const int bl = use_v ? kBW * w + 2 * p + (lane >> 5) : kBW * w + (lane & 15);
                tile[(u * kRB + rl) * kRow + bl] = rb + rl < R ? val[p] : (Real)0;
            }
        }
    };
    if (check)
        turns(std::true_type{});
    else
        turns(std::false_type{});
    __syncthreads();
    // rows (turn u, ring) of 64 consecutive angles b0 + u A / 4 + [0, 64): two values per lane
    Real* __restrict__ P = g.P + (size_t)img * R * A;
    for (int i = tid; i < 4 * kRB * (kAB / 2); i += kThreads) {
        const int row = i / (kAB / 2), col = 2 * (i % (kAB / 2));
        const int u = row / kRB, r = rb + row % kRB;
        if (r < R) {
            Pair2<Real> v;
            v.a = tile[row * kRow + col];
            v.b = tile[row * kRow + col + 1];
            *reinterpret_cast<Pair2<Real>*>(P + (size_t)r * A + u * (A / 4) + b0 + col) = v;
        }
    }
}

// Workgroups are dealt round-robin to the 8 XCDs; renumber them so that each
// XCD runs a contiguous range of (frame, band, sector) tiles: the sectors of
// a band, and neighbouring bands, then share one L2.
template <typename Real>
__global__ __launch_bounds__(kThreads) void resample_kernel(ResampleArgs<Real> g, int nb, int ns, int G) {
    __shared__ __attribute__((aligned(16))) Real tile[4 * kRB * kRow];
    const int per_xcd = (int)(gridDim.x / 8);
    const int lid = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (lid >= G) return;
    const int per_img = nb * ns;
    const int img = lid / per_img, rem = lid % per_img;
    resample_tile<Real>(g, img, (rem / ns) * kRB, (rem % ns) * kAB, tile);
}

template <typename Real>
hipError_t launch_real(const zm_plan_s* p, const void* src, long long stride, int batch, void* P, hipStream_t s) {
    ResampleArgs<Real> g;
    g.src = (const Real*)src;
    g.src_stride = stride;
    g.H = p->H;
    g.W = p->W;
    g.R = p->R;
    g.A = p->A;
    g.cx = p->cx;
    g.cy = p->cy;
    g.safe_s = fmin(p->cx, p->cy) - 1e-6;
    g.spx = p->d_spx;
    g.trig = p->d_trig;
    g.P = (Real*)P;
    const int nb = (p->R + kRB - 1) / kRB, ns = (p->A / 4) / kAB;
    const long long G = (long long)nb * ns * batch;
    if (G > 0x7fffff00ll) return hipErrorInvalidValue;
    const int G8 = (int)((G + 7) / 8 * 8);
    hipLaunchKernelGGL(resample_kernel<Real>, dim3(G8), dim3(kThreads), 0, s, g, nb, ns, (int)G);
    return hipGetLastError();
}

}  // namespace

namespace zm {

bool resample_supported(int A) { return A >= 4 * kAB && A <= 4096 && (A & (A - 1)) == 0; }

hipError_t launch_resample(const zm_plan_s* p, const void* img, long long stride, int batch, void* P, hipStream_t s) {
    if (!resample_supported(p->A)) return hipErrorInvalidValue;
    if (p->dtype == ZM_F64) return launch_real<double>(p, img, stride, batch, P, s);
    return launch_real<float>(p, img, stride, batch, P, s);
}

}  // namespace zm
