// Fused pixel -> polar resampling and angular FFT per ring.
//
// For every ring r and every m = 0..n_max this computes the angular sum of
// eq. (1) on the uniform angle grid,
//     F_r[m] = sum_{a=0}^{A-1} f^(rho_r, theta_a) exp(-2 pi i m a / A),
// where f^ is the bilinear interpolation of the frame (Sec. 2.5) at
// x = cx + s_r cos(theta_a), y = cy - s_r sin(theta_a), s_r = rho_r D/2.
//
// Two rings form one complex sequence z = f^_ra + i f^_rb; one length-A
// transform gives both spectra.  Only 2 n_max + 1 of the A outputs are
// needed, so the transform is split as A = A1 * A2 with A2 >= n_max + 1:
//   a = a1 + A1 a2,  k = k2 + A2 k1,
//   X[k2 + A2 k1] = sum_a1 W_A1^(a1 k1) W_A^(a1 k2) Y_a1[k2],
//   Y_a1 = length-A2 DFT of x[a1 + A1 a2] over a2,
// and only k1 = 0 (bins 0..n_max) and k1 = A1 - 1 (bins A - n_max..A - 1)
// are formed.  Each length-A2 DFT is a radix-16 pass in registers followed
// by a radix-Q pass (A2 = 16 Q) after one LDS exchange.
//
// Work decomposition: a workgroup owns 2P consecutive rings of one frame
// (P = 2 at A = 4096; at least 16 rings for small A, run P pairs per round).
// A round first gathers its 2P rings into LDS with lane maps that keep every
// wave instruction on a small 2-D patch of the frame and every group of 4
// lanes on neighbouring pixels of one row, then A/16 threads per pair run
// the transform, each holding 16 points.  Sample angles use exact quarter-turn rotations of first-quadrant
// angles.  Twiddles come from small LDS tables; the outputs go straight to
// the ring-tile-blocked spectrum layout described at the kernel.
#include <hip/hip_runtime.h>

#include "fft_body.h"
#include "stage_body.h"

namespace {

using namespace zmk;

constexpr int kWgSize = 512;

// Staged variant (FP32 frames, A = 4096): one round of 2P rings per
// workgroup of kStageWg threads, windows from the plan.
constexpr int kStageWg = 1024;

template <int A2>
hipError_t launch_staged(const zm_plan_s* p, const void* src, long long stride, int batch, void* F, float* fmax,
                         hipStream_t s) {
    constexpr int A = 4096;
    using SS = StageShape<A, A2, kStageWg>;
    const int gx = p->Rp / (2 * SS::P);
    const int G = gx * batch;
    const int G8 = (G + 7) / 8 * 8;
    FftArgs<float> g;
    g.src = (const float*)src;
    g.src_stride = stride;
    g.H = p->H;
    g.W = p->W;
    g.cx = p->cx;
    g.cy = p->cy;
    g.safe_s = fmin(p->cx, p->cy) - 1e-6;
    g.R = p->R;
    g.Rp = p->Rp;
    g.M = p->n_max + 1;
    g.from_polar = 0;
    g.spx = p->d_spx;
    g.trig = p->d_trig;
    g.tw = (const float*)p->d_tw;
    g.F = (float*)F;
    g.fmaxbuf = fmax;
    StageArgs sa;
    sa.win = (const StageWin*)p->d_stage_win;
    sa.rows = p->d_stage_rows;
    sa.vec4 = (p->W % 4 == 0 && stride % 4 == 0 && ((uintptr_t)src & 15) == 0) ? 1 : 0;
    hipLaunchKernelGGL((polar_fft_staged_kernel<A, A2, kStageWg>), dim3(G8), dim3(kStageWg), 0, s, g, sa, gx, G);
    return hipGetLastError();
}

hipError_t dispatch_staged(const zm_plan_s* p, const void* src, long long stride, int batch, void* F, float* fmax,
                           hipStream_t s) {
    switch (p->A2) {
        case 16: return launch_staged<16>(p, src, stride, batch, F, fmax, s);
        case 32: return launch_staged<32>(p, src, stride, batch, F, fmax, s);
        case 64: return launch_staged<64>(p, src, stride, batch, F, fmax, s);
        case 128: return launch_staged<128>(p, src, stride, batch, F, fmax, s);
        case 256: return launch_staged<256>(p, src, stride, batch, F, fmax, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename Real, int A, int A2>
hipError_t launch_one(const zm_plan_s* p, const void* src, long long stride, int batch, void* F, float* fmax,
                      int from_polar, hipStream_t s) {
    // one round of 2P rings per workgroup: the rings that share cache lines
    // are then gathered by concurrently running workgroups
    using S = FftShape<Real, A, kWgSize, 1>;
    const int gx = p->Rp / (2 * S::PAIRS);
    const int G = gx * batch;
    const int G8 = (G + 7) / 8 * 8;
    FftArgs<Real> g;
    g.src = (const Real*)src;
    g.src_stride = stride;
    g.H = p->H;
    g.W = p->W;
    g.cx = p->cx;
    g.cy = p->cy;
    g.safe_s = fmin(p->cx, p->cy) - 1e-6;
    g.R = p->R;
    g.Rp = p->Rp;
    g.M = p->n_max + 1;
    g.from_polar = from_polar;
    g.spx = p->d_spx;
    g.trig = p->d_trig;
    g.tw = (const Real*)p->d_tw;
    g.F = (Real*)F;
    g.fmaxbuf = fmax;
    hipLaunchKernelGGL((polar_fft_kernel<Real, A, A2, kWgSize, 1>), dim3(G8), dim3(S::NTHR), 0, s, g, gx, G);
    return hipGetLastError();
}

template <typename Real, int A>
hipError_t dispatch_a2(const zm_plan_s* p, const void* src, long long stride, int batch, void* F, float* fmax,
                       int from_polar, hipStream_t s) {
    switch (p->A2) {
        case 16:
            if constexpr (A >= 32) return launch_one<Real, A, 16>(p, src, stride, batch, F, fmax, from_polar, s);
            break;
        case 32:
            if constexpr (A >= 64) return launch_one<Real, A, 32>(p, src, stride, batch, F, fmax, from_polar, s);
            break;
        case 64:
            if constexpr (A >= 128) return launch_one<Real, A, 64>(p, src, stride, batch, F, fmax, from_polar, s);
            break;
        case 128:
            if constexpr (A >= 256) return launch_one<Real, A, 128>(p, src, stride, batch, F, fmax, from_polar, s);
            break;
        case 256:
            if constexpr (A >= 512 && RealTraits<Real>::kMaxA2 >= 256)
                return launch_one<Real, A, 256>(p, src, stride, batch, F, fmax, from_polar, s);
            break;
        default:
            break;
    }
    return hipErrorInvalidValue;
}

template <typename Real>
hipError_t dispatch_a(const zm_plan_s* p, const void* src, long long stride, int batch, void* F, float* fmax,
                      int from_polar, hipStream_t s) {
    switch (p->A) {
        case 32: return dispatch_a2<Real, 32>(p, src, stride, batch, F, fmax, from_polar, s);
        case 64: return dispatch_a2<Real, 64>(p, src, stride, batch, F, fmax, from_polar, s);
        case 128: return dispatch_a2<Real, 128>(p, src, stride, batch, F, fmax, from_polar, s);
        case 256: return dispatch_a2<Real, 256>(p, src, stride, batch, F, fmax, from_polar, s);
        case 512: return dispatch_a2<Real, 512>(p, src, stride, batch, F, fmax, from_polar, s);
        case 1024: return dispatch_a2<Real, 1024>(p, src, stride, batch, F, fmax, from_polar, s);
        case 2048:
            if constexpr (RealTraits<Real>::kMaxA >= 2048)
                return dispatch_a2<Real, 2048>(p, src, stride, batch, F, fmax, from_polar, s);
            break;
        case 4096:
            if constexpr (RealTraits<Real>::kMaxA >= 4096)
                return dispatch_a2<Real, 4096>(p, src, stride, batch, F, fmax, from_polar, s);
            break;
        default:
            break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

namespace zm {

hipError_t launch_polar_fft(const zm_plan_s* p, const void* img, long long stride, int batch, void* F,
                            float* fmax, int from_polar, hipStream_t s) {
    if (p->dtype == ZM_F64) return dispatch_a<double>(p, img, stride, batch, F, fmax, from_polar, s);
    if (p->stage_nthr == kStageWg && p->A == 4096 && !from_polar)
        return dispatch_staged(p, img, stride, batch, F, fmax, s);
    return dispatch_a<float>(p, img, stride, batch, F, fmax, from_polar, s);
}

bool polar_fft_supported(zm_dtype dt, int A, int A2) {
    const int maxA = (dt == ZM_F64) ? RealTraits<double>::kMaxA : RealTraits<float>::kMaxA;
    const int maxA2 = (dt == ZM_F64) ? RealTraits<double>::kMaxA2 : RealTraits<float>::kMaxA2;
    return A >= 32 && A <= maxA && (A & (A - 1)) == 0 && A2 >= 16 && A2 <= maxA2 && A2 * 2 <= A;
}

}  // namespace zm
