// Fused resample + angular FFT with the frame staged through LDS (FP32
// frames, large A).  Same samples and the same transform as polar_fft_tile
// (bit for bit); what changes is how the bilinear taps reach the samples.
//
// A workgroup of NTHR threads owns one round of 2P rings (P = NTHR / NT ring
// pairs, NT = A / 16 threads per pair) and walks the circle in 16 sectors of
// NT consecutive angles.  Thread t of pair f computes, in sector j, the
// samples of rings 2f and 2f + 1 at angle t + NT j: exactly the point
// z[j] = x[t + NT j] that it feeds to the radix-16 pass, so the samples go
// straight into registers and the LDS that the transform needs later is free
// during the gather.  That LDS holds two staging buffers: while a sector is
// sampled from one, the frame pixels of the next sector are loaded into
// registers with 16-byte row loads and then written to the other.
//
// What a sector reads is fixed by the plan's geometry, not by the frame, so
// the plan lays it out once on the host (by the same coordinate arithmetic,
// sample_pos): for every tap row, the run of 4-pixel chunks the sector's
// taps touch (plus one pixel of margin on each side and one row above and
// below).  Staged rows sit at a uniform pitch; a per-row base offset turns
// (row, column) into an LDS index.  Chunks outside the frame stage zeros,
// which is what the bilinear interpolation takes for pixels outside it.
#pragma once

#include <algorithm>
#include <vector>

#include "fft_body.h"

namespace zmk {

// Staging window of one (round, sector): rows imin .. imin + nrows - 1,
// at most cmax chunks per row (LDS pitch 4 cmax floats), row entries from
// rowoff in the row table, magic = floor(2^32 / cmax) + 1 (exact division
// of a chunk index by cmax below 2^16).
struct StageWin {
    int imin, nrows, cmax, rowoff;
    unsigned magic;
    int pad0, pad1, pad2;
};

// Row entry: (first column of the run << 8) | number of 4-pixel chunks.
__host__ __device__ inline int stage_row_entry(int xs, int nchunks) { return (int)((unsigned)xs << 8) | nchunks; }

template <int A, int A2, int NTHR>
struct StageShape {
    using L = FftLds<float, A, A2, NTHR, 1>;
    static constexpr int NT = L::NT, P = L::P;
    static_assert(P * NT == NTHR, "one round of P pairs per workgroup");
    static constexpr int kMaxRows = 512;  // staged rows per window
    // two staging buffers and two row-base tables inside the transform's LDS
    static constexpr int kCap = (int)(((size_t)P * L::XSZ * 2 - 2 * kMaxRows) / 2 / 4 * 4);
    static constexpr int kLoads = 5;      // 16-byte chunks per thread per window
};

struct StageArgs {
    const StageWin* win;  // [round][16]
    const int* rows;      // row entries
    int vec4;             // frame rows and base allow 16-byte loads
};

// Staging windows of the staged resample + FFT for workgroups of NTHR
// threads (see stage_body.h): for every round of 2P rings and each of the 16
// sectors of A / 16 angles, the taps of every sample are located with the
// kernel's own coordinate arithmetic; each tap row gets the run of 4-pixel
// chunks covering its taps plus one pixel on either side, and the window one
// extra row above and below.  Returns false (staging off for the plan) when
// a window exceeds the kernel's staging buffer.
template <int A, int A2, int NTHR>
inline bool stage_windows(int H, int W, int R, int Rp, double cx, double cy, const std::vector<double>& spx,
                   const std::vector<double>& trig, std::vector<StageWin>& wins, std::vector<int>& rows) {
    using SS = StageShape<A, A2, NTHR>;
    constexpr int NT = SS::NT, P = SS::P, kStep = A / 32;
    const int rounds = Rp / (2 * P);
    wins.assign((size_t)rounds * 16, StageWin{0, 0, 2, 0, 0u, 0, 0, 0});
    rows.clear();
    std::vector<int> lo, hi;
    for (int k = 0; k < rounds; ++k) {
        const int r0 = k * 2 * P;
        if (r0 >= R) continue;
        for (int j = 0; j < 16; ++j) {
            const int u = j / 4;
            int rmin = 1 << 30, rmax = -(1 << 30);
            // pass 1: row range; pass 2: column runs
            for (int pass = 0; pass < 2; ++pass) {
                for (int r = r0; r < std::min(r0 + 2 * P, R); ++r) {
                    for (int t = 0; t < NT; ++t) {
                        const int b = t + NT * (j & 3);
                        double cb, sb;
                        rotate_pair(trig[2 * (b % kStep)], trig[2 * (b % kStep) + 1], trig[2 * kStep * (b / kStep)],
                                         trig[2 * kStep * (b / kStep) + 1], cb, sb);
                        const TapPos<float> tp =
                            sample_pos<float>(cx, cy, W, H, spx[r], cb, sb, u);
                        const int i0 = tp.y.i, j0 = tp.x.i;
                        if (pass == 0) {
                            rmin = std::min(rmin, i0);
                            rmax = std::max(rmax, i0 + 1);
                        } else {
                            for (int d = 0; d < 2; ++d) {
                                const int q = i0 + d - (rmin - 1);
                                lo[q] = std::min(lo[q], j0 - 1);
                                hi[q] = std::max(hi[q], j0 + 2);
                            }
                        }
                    }
                }
                if (pass == 0) {
                    const int n = rmax - rmin + 3;
                    lo.assign(n, 1 << 30);
                    hi.assign(n, -(1 << 30));
                }
            }
            const int nrows = rmax - rmin + 3;
            int cmax = 2;
            const int off = (int)rows.size();
            for (int q = 0; q < nrows; ++q) {
                if (lo[q] > hi[q]) {
                    rows.push_back(stage_row_entry(0, 0));
                    continue;
                }
                const int xs = lo[q] >= 0 ? (lo[q] & ~3) : -((-lo[q] + 3) & ~3);
                const int nch = (hi[q] - xs) / 4 + 1;
                cmax = std::max(cmax, nch);
                rows.push_back(stage_row_entry(xs, nch));
            }
            if (nrows > SS::kMaxRows || nrows * 4 * cmax > SS::kCap || nrows * cmax > SS::kLoads * NTHR || cmax > 255)
                return false;
            StageWin& w = wins[(size_t)k * 16 + j];
            w.imin = rmin - 1;
            w.nrows = nrows;
            w.cmax = cmax;
            w.rowoff = off;
            w.magic = (unsigned)((1ull << 32) / (unsigned)cmax + 1);
        }
    }
    return true;
}

template <int A, int A2, int NTHR>
__device__ __forceinline__ void polar_fft_staged_tile(const FftArgs<float>& g, const StageArgs& sa, int img, int tile,
                                                      char* smem) {
    using C = cplx<float>;
    using L = FftLds<float, A, A2, NTHR, 1>;
    using SS = StageShape<A, A2, NTHR>;
    constexpr int NT = L::NT, P = L::P, XSZ = L::XSZ, NLO = L::NLO, NHI = L::NHI, A1 = L::A1;
    constexpr int CAP = SS::kCap, MAXR = SS::kMaxRows, NL = SS::kLoads;
    const int H = g.H, W = g.W, R = g.R, Rp = g.Rp, M = g.M;
    const double cx = g.cx, cy = g.cy;

    C* xbuf = reinterpret_cast<C*>(smem);
    C* tA2 = xbuf + P * XSZ;
    C* tLo = tA2 + A2;
    C* tHi = tLo + NLO;
    C* w3 = tHi + NHI;
    float* red = reinterpret_cast<float*>(w3 + A1);
    float* sbuf = reinterpret_cast<float*>(xbuf);   // [2][CAP]
    int* sbase = reinterpret_cast<int*>(sbuf + 2 * CAP);  // [2][MAXR]

    const int tid = threadIdx.x;
    const int f = tid / NT;
    const int t = tid % NT;
    const int r0 = tile * (2 * P);
    const int nRT = Rp / zm::kRingTile;
    const C* twc = reinterpret_cast<const C*>(g.tw);
    float* Fimg = g.F + (size_t)img * nRT * M * 2 * zm::kRingTile;

    if (r0 >= R) {  // padding rings R..Rp-1 are zero
        for (int e = tid; e < M * 2 * 2 * P; e += NTHR) {
            const int row = e / (2 * P), i = e % (2 * P);
            const int r = r0 + i;
            Fimg[((size_t)(r / zm::kRingTile) * M * 2 + row) * zm::kRingTile + (r % zm::kRingTile)] = 0.f;
        }
        return;
    }
    for (int i = tid; i < A2; i += NTHR) tA2[i] = twc[i * A1];
    for (int i = tid; i < NLO; i += NTHR) tLo[i] = twc[i < A ? i : 0];
    for (int i = tid; i < NHI; i += NTHR) tHi[i] = twc[(i * NLO) % A];
    for (int i = tid; i < A1; i += NTHR) w3[i] = twc[i * A2];

    const float* __restrict__ frame = g.src + (size_t)img * (size_t)g.src_stride;
    const StageWin* __restrict__ win = sa.win + (size_t)tile * 16;
    const int* __restrict__ rowtab = sa.rows;
    const int vec4 = sa.vec4;

    const int ra = r0 + 2 * f, rb = ra + 1;
    const bool ina = ra < R, inb = rb < R;
    const double sra = ina ? g.spx[ra] : 0.0, srb = inb ? g.spx[rb] : 0.0;
    // base angle b = t + NT (j mod 4) < A / 4; with step A / 32 = NT / 2,
    // b mod step = t mod (NT / 2) for every sector, b div step = 2 (j mod 4) + t div (NT / 2)
    constexpr int kStep = A / 32;
    static_assert(2 * kStep == NT, "sector base angles step by A / 32");
    const double c0 = g.trig[2 * (t % kStep)], s0 = g.trig[2 * (t % kStep) + 1];
    const int half = t / kStep;

    float4 stg[NL];
    int srow[NL], sk[NL], sxs[NL];
    // loads of window j into registers (16-byte row chunks, zeros outside the frame)
    auto issue = [&](int j) {
        const StageWin w = win[j];
        const int total = w.nrows * w.cmax;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int c = tid + NTHR * l;
            srow[l] = -1;
            stg[l] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < total) {
                const int row = (int)__umulhi((unsigned)c, w.magic);
                const int k = c - row * w.cmax;
                const int e = rowtab[w.rowoff + row];
                const int xs = e >> 8, n = e & 255;
                srow[l] = row;
                sk[l] = k;
                sxs[l] = xs;
                if (k < n) {
                    const int gy = w.imin + row, gx = xs + 4 * k;
                    if ((unsigned)gy < (unsigned)H) {
                        const float* rp = frame + (size_t)gy * W;
                        if (gx >= 0 && gx + 3 < W) {
                            if (vec4) {
                                stg[l] = *reinterpret_cast<const float4*>(rp + gx);
                            } else {
                                stg[l] = make_float4(rp[gx], rp[gx + 1], rp[gx + 2], rp[gx + 3]);
                            }
                        } else {
                            float v[4];
#pragma unroll
                            for (int d = 0; d < 4; ++d) v[d] = ((unsigned)(gx + d) < (unsigned)W) ? rp[gx + d] : 0.f;
                            stg[l] = make_float4(v[0], v[1], v[2], v[3]);
                        }
                    }
                }
            }
        }
    };
    // registers of window j -> staging buffer j & 1 and its row bases
    auto commit = [&](int j) {
        const StageWin w = win[j];
        float* buf = sbuf + (j & 1) * CAP;
        int* base = sbase + (j & 1) * MAXR;
        const int pitch = 4 * w.cmax;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            if (srow[l] >= 0) {
                const int row = srow[l], k = sk[l];
                *reinterpret_cast<float4*>(buf + row * pitch + 4 * k) = stg[l];
                if (k == 0) base[row] = row * pitch - sxs[l];
            }
        }
    };

    __syncthreads();  // twiddle tables written
    issue(0);
    commit(0);
    __syncthreads();
    C z[16];
    float vmax = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {  // unrolled: z[j] stays in registers
        if (j + 1 < 16) issue(j + 1);
        const int imin = win[j].imin;
        const float* buf = sbuf + (j & 1) * CAP;
        const int* base = sbase + (j & 1) * MAXR;
        const int u = j >> 2;
        const int bi = 2 * (j & 3) + half;
        double cb, sb;
        rotate_pair(c0, s0, g.trig[2 * kStep * bi], g.trig[2 * kStep * bi + 1], cb, sb);
        float v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bool in = h ? inb : ina;
            v[h] = 0.f;
            if (in) {
                const TapPos<float> tp = sample_pos<float>(cx, cy, W, H, h ? srb : sra, cb, sb, u);
                const int row = tp.y.i - imin;
                const int b0 = base[row] + tp.x.i, b1 = base[row + 1] + tp.x.i;
                v[h] = bilerp(buf[b0], buf[b0 + 1], buf[b1], buf[b1 + 1], tp.x.f, tp.y.f);
            }
        }
        z[j] = C{v[0], v[1]};
        if (j + 1 < 16) commit(j + 1);
        __syncthreads();
    }
    fft_pair<float, A, A2, NTHR, 1>(z, xbuf + f * XSZ, tA2, tLo, tHi, w3, t, ra, Fimg, M, vmax);
    if (g.fmaxbuf != nullptr) {
        red[tid] = vmax;
        __syncthreads();
        for (int s = NTHR / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
            __syncthreads();
        }
        if (tid == 0) atomicMax(reinterpret_cast<unsigned*>(g.fmaxbuf) + img, __float_as_uint(red[0]));
    }
}

template <int A, int A2, int NTHR>
__global__ __launch_bounds__(NTHR) void polar_fft_staged_kernel(FftArgs<float> g, StageArgs sa, int gx, int G) {
    __shared__ __attribute__((aligned(16))) char smem[FftLds<float, A, A2, NTHR, 1>::bytes];
    const int per_xcd = (int)(gridDim.x / 8);
    const int lid = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (lid >= G) return;
    polar_fft_staged_tile<A, A2, NTHR>(g, sa, lid / gx, lid % gx, smem);
}

}  // namespace zmk
