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
// Work decomposition: a workgroup owns 16 consecutive rings (8 pairs) of one
// frame and runs P pairs per round.  Each round first gathers the 2P rings
// into LDS with a lane mapping that keeps every wave instruction on a small
// 2-D patch of the frame (and lets the rings of the round share cache
// lines), then A/16 threads per pair run the transform, each holding 16
// points.  Sample angles use exact quarter-turn rotations of first-quadrant
// angles.  Twiddles come from small LDS tables; the outputs go straight to
// the ring-tile-blocked spectrum layout described at the kernel.
#include <hip/hip_runtime.h>

#include "zm_internal.h"

namespace {

template <typename Real>
struct cplx {
    Real x, y;
};

template <typename Real>
__device__ __forceinline__ cplx<Real> operator+(cplx<Real> a, cplx<Real> b) { return {a.x + b.x, a.y + b.y}; }
template <typename Real>
__device__ __forceinline__ cplx<Real> operator-(cplx<Real> a, cplx<Real> b) { return {a.x - b.x, a.y - b.y}; }
// z * exp(-i t) with (c, s) = (cos t, sin t)
template <typename Real>
__device__ __forceinline__ cplx<Real> mulw(cplx<Real> z, Real c, Real s) {
    return {z.x * c + z.y * s, z.y * c - z.x * s};
}
// z * (-i)
template <typename Real>
__device__ __forceinline__ cplx<Real> mul_mi(cplx<Real> z) { return {z.y, -z.x}; }

// cos / sin of 2 pi p / 16 for the radix-16 internal twiddles
constexpr double kC1 = 0.92387953251128675613;  // cos(pi/8)
constexpr double kS1 = 0.38268343236508977173;  // sin(pi/8)
constexpr double kR2 = 0.70710678118654752440;  // cos(pi/4)

template <typename Real>
__device__ __forceinline__ void dft4(cplx<Real>& a, cplx<Real>& b, cplx<Real>& c, cplx<Real>& d) {
    cplx<Real> s0 = a + c, d0 = a - c, s1 = b + d, d1 = mul_mi(b - d);
    a = s0 + s1;
    c = s0 - s1;
    b = d0 + d1;
    d = d0 - d1;
}

// In-place length-N forward DFT (exp(-2 pi i j k / N)), natural order in and out.
template <typename Real, int N>
struct SmallDft;

template <typename Real>
struct SmallDft<Real, 1> {
    __device__ __forceinline__ static void run(cplx<Real>*) {}
};
template <typename Real>
struct SmallDft<Real, 2> {
    __device__ __forceinline__ static void run(cplx<Real>* z) {
        cplx<Real> t = z[0];
        z[0] = t + z[1];
        z[1] = t - z[1];
    }
};
template <typename Real>
struct SmallDft<Real, 4> {
    __device__ __forceinline__ static void run(cplx<Real>* z) { dft4(z[0], z[1], z[2], z[3]); }
};
template <typename Real>
struct SmallDft<Real, 8> {
    // j = j1 + 2 j2, k = k1 + 4 k2: length-4 DFTs over j2, twiddle W8^(j1 k1), length-2 over j1
    __device__ __forceinline__ static void run(cplx<Real>* z) {
        cplx<Real> u0[4] = {z[0], z[2], z[4], z[6]};
        cplx<Real> u1[4] = {z[1], z[3], z[5], z[7]};
        dft4(u0[0], u0[1], u0[2], u0[3]);
        dft4(u1[0], u1[1], u1[2], u1[3]);
        const Real r2 = (Real)kR2;
        u1[1] = mulw(u1[1], r2, r2);
        u1[2] = mul_mi(u1[2]);
        u1[3] = mulw(u1[3], -r2, r2);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            z[k1] = u0[k1] + u1[k1];
            z[k1 + 4] = u0[k1] - u1[k1];
        }
    }
};
template <typename Real>
struct SmallDft<Real, 16> {
    // j = j1 + 4 j2, k = k1 + 4 k2: length-4 DFTs over j2, twiddle W16^(j1 k1), length-4 over j1
    __device__ __forceinline__ static void run(cplx<Real>* z) {
#pragma unroll
        for (int j1 = 0; j1 < 4; ++j1) dft4(z[j1], z[j1 + 4], z[j1 + 8], z[j1 + 12]);
        finish(z);
    }
    // second half: z[j1 + 4 k1] = U[j1][k1] on entry, natural order on exit
    __device__ __forceinline__ static void finish(cplx<Real>* z) {
        const Real c1 = (Real)kC1, s1 = (Real)kS1, r2 = (Real)kR2;
        z[5] = mulw(z[5], c1, s1);      // W16^1
        z[9] = mulw(z[9], r2, r2);      // W16^2
        z[13] = mulw(z[13], s1, c1);    // W16^3
        z[6] = mulw(z[6], r2, r2);      // W16^2
        z[10] = mul_mi(z[10]);          // W16^4
        z[14] = mulw(z[14], -r2, r2);   // W16^6
        z[7] = mulw(z[7], s1, c1);      // W16^3
        z[11] = mulw(z[11], -r2, r2);   // W16^6
        z[15] = mulw(z[15], -c1, -s1);  // W16^9
        cplx<Real> out[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            // U[j1][k1] sits at z[j1 + 4 k1]; the length-4 DFT over j1 gives X[k1 + 4 k2]
            cplx<Real> a = z[4 * k1 + 0], b = z[4 * k1 + 1], c = z[4 * k1 + 2], d = z[4 * k1 + 3];
            dft4(a, b, c, d);
            out[k1 + 0] = a;
            out[k1 + 4] = b;
            out[k1 + 8] = c;
            out[k1 + 12] = d;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) z[i] = out[i];
    }
};

template <typename Real>
struct alignas(2 * sizeof(Real)) Pair2 {
    Real a, b;
};

template <typename Real>
struct RealTraits;
template <>
struct RealTraits<float> {
    static constexpr int kMaxA = 4096;
    static constexpr int kMaxA2 = 256;
};
template <>
struct RealTraits<double> {
    static constexpr int kMaxA = 1024;
    static constexpr int kMaxA2 = 128;  // LDS bound of the FP64 variant
};

// Bilinear sample of the frame from tap origin (j0, i0) and fractions
// (fx, fy) in [0, 1].  CHECK selects the path that treats taps outside the
// frame as 0 (tap indices are clamped before the loads, so no load leaves the
// frame); without CHECK the caller guarantees 0 <= j0 <= W-2, 0 <= i0 <= H-2.
template <typename Real, bool CHECK>
__device__ __forceinline__ Real bilinear_idx(const Real* __restrict__ img, int H, int W, int j0, int i0, Real fx,
                                             Real fy) {
    Real v00, v01, v10, v11;
    if (CHECK) {
        const int ja = min(max(j0, 0), W - 1), jb = min(max(j0 + 1, 0), W - 1);
        const int ia = min(max(i0, 0), H - 1), ib = min(max(i0 + 1, 0), H - 1);
        const bool jin0 = (unsigned)j0 < (unsigned)W, jin1 = (unsigned)(j0 + 1) < (unsigned)W;
        const bool iin0 = (unsigned)i0 < (unsigned)H, iin1 = (unsigned)(i0 + 1) < (unsigned)H;
        const Real t00 = img[(unsigned)(ia * W + ja)], t01 = img[(unsigned)(ia * W + jb)];
        const Real t10 = img[(unsigned)(ib * W + ja)], t11 = img[(unsigned)(ib * W + jb)];
        v00 = (iin0 && jin0) ? t00 : (Real)0;
        v01 = (iin0 && jin1) ? t01 : (Real)0;
        v10 = (iin1 && jin0) ? t10 : (Real)0;
        v11 = (iin1 && jin1) ? t11 : (Real)0;
    } else {
        // two rows of two adjacent taps: each row is one 8-byte load
        const Real* r0p = img + (i0 * W + j0);
        const Real* r1p = r0p + W;
        v00 = r0p[0];
        v01 = r0p[1];
        v10 = r1p[0];
        v11 = r1p[1];
    }
    const Real top = v00 + fx * (v01 - v00);
    const Real bot = v10 + fx * (v11 - v10);
    return top + fy * (bot - top);
}

// floor and fraction of a pixel coordinate
template <typename Real>
struct Coord {
    int i;
    Real f;
};
template <typename Real>
__device__ __forceinline__ Coord<Real> split_coord(double v) {
    const double fl = floor(v);
    return Coord<Real>{(int)fl, (Real)(v - fl)};
}
// K - v for integer K, from the split of v: floor = K - floor(v) - 1 and
// fraction 1 - frac(v) (a fraction of exactly 1 when v is an integer, which
// bilinear interpolation treats identically to fraction 0 one tap further).
template <typename Real>
__device__ __forceinline__ Coord<Real> mirror_coord(Coord<Real> c, int K) {
    return Coord<Real>{K - c.i - 1, (Real)1 - c.f};
}

template <int A>
struct FftShape {
    static constexpr int NT = A / 16;                          // threads per transform
    // transforms in flight: 512 threads per workgroup (two workgroups per
    // CU), at most 8 pairs per round
    static constexpr int P = (512 / NT) < 1 ? 1 : ((512 / NT) > 8 ? 8 : (512 / NT));
    static constexpr int NTHR = NT * P;                        // workgroup size
    static constexpr int PAIRS = 8;                            // ring pairs per workgroup (16 rings)
    static constexpr int ROUNDS = PAIRS / P;
    static constexpr int RPR = 2 * P;                          // rings gathered per round
};

// LDS row padding of the first exchange: consecutive lane groups of A1
// threads read rows KG*S1 complex apart; choose S1 so those groups land on
// disjoint halves of the 64 banks.
constexpr int pad_s1(int NT, int KG, int A1) {
    if (A1 >= 32) return 1;
    for (int pad = 1; pad <= 32; ++pad)
        if ((KG * (NT + pad)) % 32 == A1 % 32) return pad;
    return 1;
}

// Ring spectra layout (the projection's operand): frame b, ring tile
// rt = r / 16, bin m, part c (0 = re, 1 = im), ring r % 16:
//   F[(((b * nRT + rt) * M + m) * 2 + c) * 16 + r % 16].
// Each ring pair writes 8-byte pieces; the workgroup owns all 16 rings of a
// tile, so every 128-byte line (both parts of one m) is completed by one
// workgroup within microseconds and leaves L2 as a full line.
template <typename Real, int A, int A2>
__global__ __launch_bounds__(FftShape<A>::NTHR) __attribute__((amdgpu_waves_per_eu(4))) void polar_fft_kernel(
    const Real* __restrict__ src, long long src_stride, int H, int W, double cx, double cy, double safe_s,
    int R, int Rp, int M, int from_polar, const double* __restrict__ spx, const double* __restrict__ trig,
    const Real* __restrict__ tw, Real* __restrict__ F, float* __restrict__ fmaxbuf, int gx, int G) {
    using C = cplx<Real>;
    using S = FftShape<A>;
    constexpr int NT = S::NT, P = S::P, NTHR = S::NTHR, ROUNDS = S::ROUNDS, PAIRS = S::PAIRS;
    constexpr int A1 = A / A2;
    constexpr int Q = A2 / 16;
    constexpr int KG = 16 / Q;
    constexpr int S1 = NT + pad_s1(NT, KG, A1);
    constexpr int S2 = A1 + 1;
    constexpr int XSZ0 = (16 * S1 > A2 * S2) ? 16 * S1 : A2 * S2;
    constexpr int XSZ1 = XSZ0 > A ? XSZ0 : A;  // also holds the A gathered samples of a pair
    // pair slots are 32/P complex (mod 32) apart, so the gather's lanes
    // (rings fastest, then angles) write to distinct banks
    constexpr int SLOT = 32 / P;
    constexpr int XSZ = XSZ1 + ((SLOT - XSZ1 % 32) % 32 + 32) % 32;
    constexpr int NLO = 64;           // two-level table of W_A^x: x = 64 hi + lo
    constexpr int NHI = A / NLO > 0 ? A / NLO : 1;

    __shared__ C xbuf[P * XSZ];
    __shared__ C tA2[A2];             // W_A2^x  (= W_A^(x A1)), x < A2
    __shared__ C tLo[NLO];            // W_A^x, x < 64
    __shared__ C tHi[NHI];            // W_A^(64 x)
    __shared__ C w3[A1];              // exp(+2 pi i a1 / A1)
    __shared__ float red[NTHR];

    const int tid = threadIdx.x;
    const int f = tid / NT;  // transform slot
    const int t = tid % NT;  // thread within the transform
    const int a1 = t % A1;
    const int q = t / A1;    // phase-1 sub index; also the phase-2 k' group
    // Workgroups are dealt round-robin to the 8 XCDs; renumber them so that
    // each XCD runs a contiguous range of (frame, ring tile) work: tiles
    // running together on one XCD are radial neighbours and share L2 lines
    // (a 128-byte line spans 32 rings where the circle runs vertically).
    const int per_xcd = (int)(gridDim.x / 8);
    const int lid = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (lid >= G) return;
    const int img = lid / gx;
    const int r0 = (lid % gx) * (2 * PAIRS);
    const int nRT = Rp / zm::kRingTile;
    const C* twc = reinterpret_cast<const C*>(tw);
    Real* Fimg = F + (size_t)img * nRT * M * 2 * zm::kRingTile;

    if (r0 >= R) {  // padding rings R..Rp-1 are zero
        for (int e = tid; e < M * 2 * 2 * PAIRS; e += NTHR) {
            const int row = e / (2 * PAIRS), i = e % (2 * PAIRS);
            const int r = r0 + i;
            Fimg[((size_t)(r / zm::kRingTile) * M * 2 + row) * zm::kRingTile + (r % zm::kRingTile)] = (Real)0;
        }
        return;
    }

    // The table entry j holds (cos, sin)(2 pi j / A) = exp(+2 pi i j / A);
    // multiplying by W^j = exp(-2 pi i j / A) is mulw(z, cos, sin).
    for (int i = tid; i < A2; i += NTHR) tA2[i] = twc[i * A1];
    for (int i = tid; i < NLO; i += NTHR) tLo[i] = twc[i < A ? i : 0];
    for (int i = tid; i < NHI; i += NTHR) tHi[i] = twc[(i * NLO) % A];
    for (int i = tid; i < A1; i += NTHR) w3[i] = twc[i * A2];  // exp(+2 pi i a1/A1) = W_A1^(a1 (A1-1))

    const Real* frame = src + (size_t)img * (size_t)src_stride;
    float vmax = 0.f;

    __syncthreads();

    for (int rd = 0; rd < ROUNDS; ++rd) {
        const int pp = rd * P + f;  // ring pair within the workgroup
        const int ra = r0 + 2 * pp, rb = ra + 1;
        C* xb = xbuf + f * XSZ;
        C z[16];
        if (from_polar) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int a = t + NT * j;
                z[j].x = (ra < R) ? frame[(size_t)ra * A + a] : (Real)0;
                z[j].y = (rb < R) ? frame[(size_t)rb * A + a] : (Real)0;
            }
            __syncthreads();  // previous round's phase-3 readers are done
        } else {
            // Gather the 2P rings of this round into LDS.  Consecutive lanes
            // take consecutive rings, then consecutive angles, so one wave
            // instruction covers a compact (2P rings x 64/2P angles) patch of
            // the frame.  Each thread keeps one ring and 8 base angles in the
            // first quadrant; the other 3 quarter turns are exact rotations.
            const int ri = tid % S::RPR;
            const int ring = r0 + rd * S::RPR + ri;
            const double sr = ring < R ? spx[ring] : 0.0;
            const int last = min(r0 + rd * S::RPR + S::RPR, R) - 1;
            const bool check = (last >= r0 + rd * S::RPR) && spx[last] >= safe_s;
            Real* xf = reinterpret_cast<Real*>(xbuf + (ri >> 1) * XSZ) + (ri & 1);
            __syncthreads();  // previous round's phase-3 readers are done
#pragma unroll 2
            for (int i = 0; i < 8; ++i) {
                const int a = (tid + NTHR * i) / S::RPR;  // base angle, < A / 4
                const double c = trig[2 * a], sn = trig[2 * a + 1];
                const double pc = sr * c, ps = sr * sn;
                // the four quarter turns: x = cx + (pc, -ps, -pc, ps), y = cy - (ps, pc, -ps, -pc);
                // with 2 cx = W - 1 and 2 cy = H - 1 the negated offsets are mirrors
                const Coord<Real> xa = split_coord<Real>(cx + pc), xb2 = split_coord<Real>(cx + ps);
                const Coord<Real> yb = split_coord<Real>(cy + ps), yd = split_coord<Real>(cy + pc);
                const Coord<Real> xs[4] = {xa, mirror_coord(xb2, W - 1), mirror_coord(xa, W - 1), xb2};
                const Coord<Real> ys[4] = {mirror_coord(yb, H - 1), mirror_coord(yd, H - 1), yb, yd};
                Real val[4];
                if (!check) {
                    // every ring of the round lies inside the safe radius; rings
                    // past R (partial last round) sample the centre and are zeroed
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const Real v = bilinear_idx<Real, false>(frame, H, W, xs[u].i, ys[u].i, xs[u].f, ys[u].f);
                        val[u] = ring < R ? v : (Real)0;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        val[u] = ring < R ? bilinear_idx<Real, true>(frame, H, W, xs[u].i, ys[u].i, xs[u].f, ys[u].f)
                                          : (Real)0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) xf[2 * (a + u * (A / 4))] = val[u];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 16; ++j) z[j] = xb[t + NT * j];
        }
        SmallDft<Real, 16>::run(z);
        // then W_A2^(q k')
#pragma unroll
        for (int k = 1; k < 16; ++k) {
            const C w = tA2[(q * k) % A2];
            z[k] = mulw(z[k], w.x, w.y);
        }
        __syncthreads();  // all reads of the gathered samples are done
#pragma unroll
        for (int k = 0; k < 16; ++k) xb[k * S1 + t] = z[k];
        __syncthreads();
        // phase 2: for k' in this thread's group, length-Q DFT over q, then W_A^(a1 k2)
        C y[KG][Q];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            const int kp = q * KG + kk;
#pragma unroll
            for (int qq = 0; qq < Q; ++qq) y[kk][qq] = xb[kp * S1 + a1 + A1 * qq];
            SmallDft<Real, Q>::run(y[kk]);
#pragma unroll
            for (int k2 = 0; k2 < Q; ++k2) {
                const int x = a1 * (kp + 16 * k2);  // < A
                const C h = tHi[x / NLO], l = tLo[x % NLO];
                const C w = C{h.x * l.x - h.y * l.y, h.x * l.y + h.y * l.x};
                y[kk][k2] = mulw(y[kk][k2], w.x, w.y);
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KG; ++kk)
#pragma unroll
            for (int k2 = 0; k2 < Q; ++k2) xb[((q * KG + kk) + 16 * k2) * S2 + a1] = y[kk][k2];
        __syncthreads();
        // phase 3: bins m (k1 = 0) and A - m (k1 = A1 - 1), then split the two rings
        const int rt = ra / zm::kRingTile, ri = ra % zm::kRingTile;
        Real* Fo = Fimg + (size_t)rt * M * 2 * zm::kRingTile + ri;
        for (int m = t; m < M; m += NT) {
            C pm = {(Real)0, (Real)0};
#pragma unroll 4
            for (int i = 0; i < A1; ++i) pm = pm + xb[m * S2 + i];
            C nm = pm;
            if (m > 0) {
                nm = C{(Real)0, (Real)0};
                const int row = A2 - m;
#pragma unroll 4
                for (int i = 0; i < A1; ++i) {
                    const C v = xb[row * S2 + i];
                    const C w = w3[i];
                    nm.x += v.x * w.x - v.y * w.y;
                    nm.y += v.x * w.y + v.y * w.x;
                }
            }
            // ring a: (X[m] + conj X[A-m]) / 2 ; ring b: (X[m] - conj X[A-m]) / (2 i)
            const Real fax = (Real)0.5 * (pm.x + nm.x), fay = (Real)0.5 * (pm.y - nm.y);
            const Real fbx = (Real)0.5 * (pm.y + nm.y), fby = (Real)0.5 * (nm.x - pm.x);
            vmax = fmaxf(vmax, fmaxf(fmaxf((float)fabs((double)fax), (float)fabs((double)fay)),
                                     fmaxf((float)fabs((double)fbx), (float)fabs((double)fby))));
            Real* o = Fo + (size_t)m * 2 * zm::kRingTile;  // ri even: 2-element aligned
            *reinterpret_cast<Pair2<Real>*>(o) = Pair2<Real>{fax, fbx};
            *reinterpret_cast<Pair2<Real>*>(o + zm::kRingTile) = Pair2<Real>{fay, fby};
        }
    }
    if (fmaxbuf != nullptr) {
        red[tid] = vmax;
        __syncthreads();
        for (int s = NTHR / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
            __syncthreads();
        }
        if (tid == 0) atomicMax(reinterpret_cast<unsigned*>(fmaxbuf) + img, __float_as_uint(red[0]));
    }
}

template <typename Real, int A, int A2>
hipError_t launch_one(const zm_plan_s* p, const void* src, long long stride, int batch, void* F, float* fmax,
                      int from_polar, hipStream_t s) {
    using S = FftShape<A>;
    const int gx = p->Rp / (2 * S::PAIRS);
    const int G = gx * batch;
    const int G8 = (G + 7) / 8 * 8;
    const double safe_s = fmin(p->cx, p->cy) - 1e-6;
    hipLaunchKernelGGL((polar_fft_kernel<Real, A, A2>), dim3(G8), dim3(S::NTHR), 0, s, (const Real*)src, stride,
                       p->H, p->W, p->cx, p->cy, safe_s, p->R, p->Rp, p->n_max + 1, from_polar, p->d_spx,
                       p->d_trig, (const Real*)p->d_tw, (Real*)F, fmax, gx, G);
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
    return dispatch_a<float>(p, img, stride, batch, F, fmax, from_polar, s);
}

bool polar_fft_supported(zm_dtype dt, int A, int A2) {
    const int maxA = (dt == ZM_F64) ? RealTraits<double>::kMaxA : RealTraits<float>::kMaxA;
    const int maxA2 = (dt == ZM_F64) ? RealTraits<double>::kMaxA2 : RealTraits<float>::kMaxA2;
    return A >= 32 && A <= maxA && (A & (A - 1)) == 0 && A2 >= 16 && A2 <= maxA2 && A2 * 2 <= A;
}

}  // namespace zm
