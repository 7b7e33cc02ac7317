// Device bodies of the fused resample + angular FFT (see polar_fft.hip for
// the method); shared by the standalone kernels and the persistent batch
// kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "zm_internal.h"

namespace zmk {

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

// Bilinear interpolation of the taps (v00, v01) of row i0 and (v10, v11) of
// row i0 + 1 at fractions (fx, fy); every gather path uses this expression.
template <typename Real>
__device__ __forceinline__ Real bilerp(Real v00, Real v01, Real v10, Real v11, Real fx, Real fy) {
    const Real top = v00 + fx * (v01 - v00);
    const Real bot = v10 + fx * (v11 - v10);
    return top + fy * (bot - top);
}

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
        // two rows of two adjacent taps: each row is one 8-byte load, addressed
        // by a 32-bit byte offset from the frame (so the load takes the frame
        // base from scalar registers and one 32-bit offset per lane; frames
        // are below 2^31 bytes)
        const char* base = reinterpret_cast<const char*>(img);
        const Real* r0p = reinterpret_cast<const Real*>(base + (unsigned)((i0 * W + j0) * (int)sizeof(Real)));
        const Real* r1p = reinterpret_cast<const Real*>(base + (unsigned)((i0 * W + j0 + W) * (int)sizeof(Real)));
        v00 = r0p[0];
        v01 = r0p[1];
        v10 = r1p[0];
        v11 = r1p[1];
    }
    return bilerp(v00, v01, v10, v11, fx, fy);
}

// floor and fraction of a pixel coordinate
template <typename Real>
struct Coord {
    int i;
    Real f;
};
template <typename Real>
__host__ __device__ __forceinline__ Coord<Real> split_coord(double v) {
    const double fl = floor(v);
    return Coord<Real>{(int)fl, (Real)(v - fl)};
}
// K - v for integer K, from the split of v: floor = K - floor(v) - 1 and
// fraction 1 - frac(v) (a fraction of exactly 1 when v is an integer, which
// bilinear interpolation treats identically to fraction 0 one tap further).
template <typename Real>
__host__ __device__ __forceinline__ Coord<Real> mirror_coord(Coord<Real> c, int K) {
    return Coord<Real>{K - c.i - 1, (Real)1 - c.f};
}

// (cos, sin) of the base angle 2 pi b / A, b < A / 4: the table pair of
// b mod (A / 32) rotated by the table pair of (A / 32) floor(b / (A / 32)),
// one rounded product each (written with explicit FMAs, so every gather
// path, and the host's window planning, forms the same bits).
__host__ __device__ __forceinline__ void rotate_pair(double c0, double s0, double ci, double si, double& c, double& s) {
    c = fma(c0, ci, -(s0 * si));
    s = fma(s0, ci, c0 * si);
}

// Tap origin (row i, column j) and fractions of the sample at radius sr
// (pixels) and angle b + u A / 4, with (cb, sb) the pair of base angle b:
// x = cx + sr (cb, -sb, -cb, sb)[u], y = cy - sr (sb, cb, -sb, -cb)[u].
// The negated offsets are mirrors of cx + sr c and cy + sr s (2 cx = W - 1,
// 2 cy = H - 1), so the four quarter turns of one base angle sit exactly on
// rotated pixel positions.
template <typename Real>
struct TapPos {
    Coord<Real> x, y;
};
template <typename Real>
__host__ __device__ __forceinline__ TapPos<Real> sample_pos(double cx, double cy, int W, int H, double sr, double cb,
                                                            double sb, int u) {
    const double c1 = (u & 1) ? sb : cb;
    const double c2 = (u & 1) ? cb : sb;
    Coord<Real> X = split_coord<Real>(fma(sr, c1, cx));
    Coord<Real> Y = split_coord<Real>(fma(sr, c2, cy));
    if (u == 1 || u == 2) X = mirror_coord(X, W - 1);
    if (u == 0 || u == 1) Y = mirror_coord(Y, H - 1);
    return TapPos<Real>{X, Y};
}

template <typename Real>
struct FftArgs {
    const Real* src;       // frames (or polar images with from_polar)
    long long src_stride;  // elements between frames
    int H, W;
    double cx, cy, safe_s;  // disk centre; rings with s_r < safe_s never touch the frame edge
    int R, Rp, M, from_polar;
    const double* spx;     // ring radius in pixels, R
    const double* trig;    // (cos, sin)(2 pi a / A), FP64
    const Real* tw;        // (cos, sin)(2 pi a / A), compute precision
    Real* F;               // spectra, ring-tile-blocked layout
    float* fmaxbuf;        // per-frame max |F| (FP16 split) or null
};

template <typename Real, int A, int WG = 512, int TP = 8>
struct FftShape {
    static constexpr int NT = A / 16;  // threads per transform
    // transforms (ring pairs) in flight: WG threads per workgroup for FP32
    // with A >= WG, at most 8 transforms otherwise
    static constexpr bool kWide = A >= WG && sizeof(Real) == 4;
    static constexpr int P = kWide ? WG / NT : ((WG / NT) > 8 ? 8 : (WG / NT));
    static constexpr int NTHR = NT * P;               // workgroup size
    static constexpr int PAIRS = P > TP ? P : TP;     // ring pairs per workgroup
    static constexpr int ROUNDS = PAIRS / P;
    static constexpr int RPR = 2 * P;                 // rings gathered per round
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
template <typename Real, int A, int A2, int WG = 512, int TP = 8>
struct FftLds {
    using S = FftShape<Real, A, WG, TP>;
    static constexpr int NT = S::NT, P = S::P, NTHR = S::NTHR;
    static constexpr int A1 = A / A2;
    static constexpr int Q = A2 / 16;
    static constexpr int KG = 16 / Q;
    static constexpr int S1 = NT + pad_s1(NT, KG, A1);
    // second exchange row stride: padded against bank conflicts, except for
    // A1 <= 4, where the padding would cost 25 % or more of the buffer
    static constexpr int S2 = A1 <= 4 ? A1 : A1 + 1;
    static constexpr int XSZ0 = (16 * S1 > A2 * S2) ? 16 * S1 : A2 * S2;
    static constexpr int XSZ1 = XSZ0 > A ? XSZ0 : A;  // also holds the A gathered samples of a pair
    // pair slots are 32/P complex (mod 32) apart, so the gather's lanes
    // (rings fastest, then angles) write to distinct banks
    static constexpr int SLOT = 32 / P > 0 ? 32 / P : 1;
    static constexpr int XSZ = XSZ1 + ((SLOT - XSZ1 % 32) % 32 + 32) % 32;
    static constexpr int NLO = 64;  // two-level table of W_A^x: x = 64 hi + lo
    static constexpr int NHI = A / NLO > 0 ? A / NLO : 1;
    // xbuf[P * XSZ], tA2[A2], tLo[NLO], tHi[NHI], w3[A1] (complex), red[NTHR] (float)
    static constexpr size_t cplx_count = (size_t)P * XSZ + A2 + NLO + NHI + A1;
    static constexpr size_t bytes = cplx_count * 2 * sizeof(Real) + (size_t)NTHR * sizeof(float);
};

// Transform of one ring pair (rings ra, ra + 1) as a function, for the
// staged gather; the direct gather includes the same block inline (see
// fft_pair_body.inc).  Every thread of the workgroup calls it (it holds
// barriers).
template <typename Real, int A, int A2, int WG, int TP>
__device__ __forceinline__ void fft_pair(cplx<Real> (&z)[16], cplx<Real>* xb, const cplx<Real>* tA2,
                                         const cplx<Real>* tLo, const cplx<Real>* tHi, const cplx<Real>* w3, int t,
                                         int ra, Real* Fimg, int M, float& vmax) {
    using C = cplx<Real>;
    using L = FftLds<Real, A, A2, WG, TP>;
    constexpr int NT = L::NT, A1 = L::A1, Q = L::Q, KG = L::KG, S1 = L::S1, S2 = L::S2, NLO = L::NLO;
    const int a1 = t % A1;
    const int q = t / A1;
#include "fft_pair_body.inc"
}

// One workgroup-tile of the fused resample + FFT: rings
// [tile * 2 PAIRS, (tile + 1) * 2 PAIRS) of frame img.  smem holds
// FftLds<Real, A, A2>::bytes bytes (16-byte aligned).
template <typename Real, int A, int A2, int WG = 512, int TP = 8>
__device__ __forceinline__ void polar_fft_tile(const FftArgs<Real>& g, int img, int tile, char* smem) {
    using C = cplx<Real>;
    using S = FftShape<Real, A, WG, TP>;
    using L = FftLds<Real, A, A2, WG, TP>;
    constexpr int NT = S::NT, P = S::P, NTHR = S::NTHR, ROUNDS = S::ROUNDS, PAIRS = S::PAIRS;
    constexpr int A1 = L::A1, Q = L::Q, KG = L::KG, S1 = L::S1, S2 = L::S2, XSZ = L::XSZ;
    constexpr int NLO = L::NLO, NHI = L::NHI;
    const Real* __restrict__ src = g.src;
    const long long src_stride = g.src_stride;
    const int H = g.H, W = g.W, R = g.R, Rp = g.Rp, M = g.M, from_polar = g.from_polar;
    const double cx = g.cx, cy = g.cy, safe_s = g.safe_s;
    const double* __restrict__ spx = g.spx;
    const double* __restrict__ trig = g.trig;
    Real* __restrict__ F = g.F;
    float* __restrict__ fmaxbuf = g.fmaxbuf;

    C* xbuf = reinterpret_cast<C*>(smem);
    C* tA2 = xbuf + P * XSZ;  // W_A2^x  (= W_A^(x A1)), x < A2
    C* tLo = tA2 + A2;        // W_A^x, x < 64
    C* tHi = tLo + NLO;       // W_A^(64 x)
    C* w3 = tHi + NHI;        // exp(+2 pi i a1 / A1)
    float* red = reinterpret_cast<float*>(w3 + A1);

    const int tid = threadIdx.x;
    const int f = tid / NT;  // transform slot
    const int t = tid % NT;  // thread within the transform
    const int a1 = t % A1;
    const int q = t / A1;    // phase-1 sub index; also the phase-2 k' group
    const int r0 = tile * (2 * PAIRS);
    const int nRT = Rp / zm::kRingTile;
    const C* twc = reinterpret_cast<const C*>(g.tw);
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
            // Gather the 2P rings of this round into LDS.  A wave instruction
            // covers a compact patch of 2P rings x 64/2P consecutive angles.
            // The texture path coalesces within groups of 4 lanes, so the
            // lanes of a group should read neighbouring pixels of one row.
            // Two lane maps cover the same patch: 4 consecutive rings at one
            // angle ("V", spread along the radius) and 4 consecutive angles of
            // one ring ("H", spread along the ring).  At angle phi from the x
            // axis a V group spans rows in proportion to dr sin(phi) and an H
            // group to ds cos(phi), with dr the ring step and ds = 2 pi r / A
            // the arc step, so V is used where tan(phi) < ds / dr.  Each
            // thread works on base angles in the first quadrant; the other 3
            // quarter turns are exact rotations: turns 0, 2 sit at angle phi =
            // base angle from the x axis, turns 1, 3 at its complement.
            const int rbase = r0 + rd * S::RPR;
            const int last = min(rbase + S::RPR, R) - 1;
            const bool check = (last >= rbase) && spx[last] >= safe_s;
            const int ri_v = tid % S::RPR;
            const double sr_v = rbase + ri_v < R ? spx[rbase + ri_v] : 0.0;
            Real* xf_v = reinterpret_cast<Real*>(xbuf + (ri_v >> 1) * XSZ) + (ri_v & 1);
            // With NTHR / 4 a multiple of RPR the H ring of a thread is the same
            // in every iteration, and the H angles of a wave are its V angles:
            // radius and (cos, sin) are passed across lanes (lane
            // RPR * (lane / RPR) + ri holds ring ri).
            constexpr bool kHFixed = (NTHR / 4) % S::RPR == 0 && S::RPR <= 16;
            const int ri_h0 = (tid >> 2) % S::RPR;
            const double sr_h0 = kHFixed ? __shfl(sr_v, ((tid & 63) & ~(S::RPR - 1)) + ri_h0, 64)
                                         : (rbase + ri_h0 < R ? spx[rbase + ri_h0] : 0.0);
            // Iteration i holds base angles in [i, i + 1) pi / 16; kv counts
            // the iterations whose mid angle has tan below ds / dr at this
            // round's first ring.  Turns 0, 2 of iteration i use V when
            // i < kv, turns 1, 3 when 7 - i < kv.  kv = 4 is the octant split,
            // the only choice without kHFixed: the two maps then cover the
            // same samples over iterations 0..3 and 4..7 but not per iteration.
            int kv = 4;
            if (kHFixed && R > 1 && rbase < R) {
                const int rn = rbase + 1 < R ? rbase + 1 : rbase - 1;
                const double dr = fabs(spx[rn] - spx[rbase]);
                const double ratio = 6.283185307179586 * spx[rbase] / ((double)A * dr);
                // tan(pi (2 j + 1) / 32), j = 0..7
                constexpr double kTanMid[8] = {0.09849140335716425, 0.3033466836073424, 0.5345111359507916,
                                               0.8206787908286602,  1.2185035255879764, 1.8708684117893888,
                                               3.296558208938321,   10.153170387608842};
                kv = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) kv += kTanMid[j] < ratio ? 1 : 0;
            }
            // The V base angle advances by NTHR / RPR = A / 32 per iteration:
            // one (cos, sin) per thread, rotated by the wave-uniform (cos, sin)
            // of 2 pi i / 32 (one rounded product per iteration, no recurrence).
            constexpr int kStep = NTHR / S::RPR;
            static_assert(NTHR % S::RPR == 0 && 32 * kStep == A, "base angles step by A / 32");
            const int a_v0 = tid / S::RPR;
            const double c0 = trig[2 * a_v0], s0 = trig[2 * a_v0 + 1];
            __syncthreads();  // previous round's phase-3 readers are done
#pragma unroll 2
            for (int i = 0; i < 8; ++i) {
                const int a_v = a_v0 + kStep * i;  // base angle, < A / 4
                const int rest = (tid + NTHR * i) >> 2;
                const int ri_h = kHFixed ? ri_h0 : rest % S::RPR;
                const int a_h = (rest / S::RPR) * 4 + (tid & 3);
                const double sr_h = kHFixed ? sr_h0 : (rbase + ri_h < R ? spx[rbase + ri_h] : 0.0);
                const double ci = trig[2 * kStep * i], si = trig[2 * kStep * i + 1];
                double cv, sv;
                rotate_pair(c0, s0, ci, si, cv, sv);
                double ch, sh;
                if constexpr (kHFixed) {
                    // lane RPR * k of the wave holds V angle (first V angle of the wave) + k
                    const int a_w0 = (tid - (tid & 63) + NTHR * i) / S::RPR;
                    const int src = (tid & ~63) + S::RPR * (a_h - a_w0);
                    ch = __shfl(cv, src & 63, 64);
                    sh = __shfl(sv, src & 63, 64);
                } else {
                    ch = trig[2 * a_h];
                    sh = trig[2 * a_h + 1];
                }
                // turns 0, 2 use (ring, angle) p; turns 1, 3 use q
                const bool p_v = i < kv, q_v = i >= 8 - kv;
                const int ri_p = p_v ? ri_v : ri_h, a_p = p_v ? a_v : a_h;
                const int ri_q = q_v ? ri_v : ri_h, a_q = q_v ? a_v : a_h;
                const double sr_p = p_v ? sr_v : sr_h, sr_q = q_v ? sr_v : sr_h;
                const double cp = p_v ? cv : ch, sp = p_v ? sv : sh;
                const double cq = q_v ? cv : ch, sq = q_v ? sv : sh;
                // the four quarter turns of (c, s) as in sample_pos: x = cx + (c, -s, -c, s),
                // y = cy - (s, c, -s, -c); the negated offsets are mirrors
                const Coord<Real> xa = split_coord<Real>(fma(sr_p, cp, cx)), yb = split_coord<Real>(fma(sr_p, sp, cy));
                const Coord<Real> xb2 = split_coord<Real>(fma(sr_q, sq, cx)), yd = split_coord<Real>(fma(sr_q, cq, cy));
                const Coord<Real> xs[4] = {xa, mirror_coord(xb2, W - 1), mirror_coord(xa, W - 1), xb2};
                const Coord<Real> ys[4] = {mirror_coord(yb, H - 1), mirror_coord(yd, H - 1), yb, yd};
                const bool in_p = rbase + ri_p < R, in_q = rbase + ri_q < R;
                Real val[4];
                if (!check) {
                    // every ring of the round lies inside the safe radius; rings
                    // past R (partial last round) sample the centre and are zeroed
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const Real v = bilinear_idx<Real, false>(frame, H, W, xs[u].i, ys[u].i, xs[u].f, ys[u].f);
                        val[u] = ((u & 1) ? in_q : in_p) ? v : (Real)0;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        val[u] = ((u & 1) ? in_q : in_p)
                                     ? bilinear_idx<Real, true>(frame, H, W, xs[u].i, ys[u].i, xs[u].f, ys[u].f)
                                     : (Real)0;
                }
                Real* xf_h = reinterpret_cast<Real*>(xbuf + (ri_h >> 1) * XSZ) + (ri_h & 1);
                Real* xf_p = p_v ? xf_v : xf_h;
                Real* xf_q = q_v ? xf_v : xf_h;
                xf_p[2 * a_p] = val[0];
                xf_q[2 * (a_q + A / 4)] = val[1];
                xf_p[2 * (a_p + A / 2)] = val[2];
                xf_q[2 * (a_q + 3 * (A / 4))] = val[3];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 16; ++j) z[j] = xb[t + NT * j];
        }
        {
#include "fft_pair_body.inc"
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

// Standalone launch: one workgroup per (frame, ring tile).  Workgroups are
// dealt round-robin to the 8 XCDs; renumber them so that each XCD runs a
// contiguous range of (frame, ring tile) work: tiles running together on one
// XCD are radial neighbours and share L2 lines (a 128-byte line spans 32
// rings where the circle runs vertically).
template <typename Real, int A, int A2, int WG = 512, int TP = 8>
__global__ __launch_bounds__((FftShape<Real, A, WG, TP>::NTHR)) __attribute__((amdgpu_waves_per_eu(4))) void polar_fft_kernel(
    FftArgs<Real> g, int gx, int G) {
    __shared__ __attribute__((aligned(16))) char smem[FftLds<Real, A, A2, WG, TP>::bytes];
    const int per_xcd = (int)(gridDim.x / 8);
    const int lid = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (lid >= G) return;
    polar_fft_tile<Real, A, A2, WG, TP>(g, lid / gx, lid % gx, smem);
}

}  // namespace zmk
