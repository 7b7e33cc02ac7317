// Device body of the radial projection on MFMA (see project.hip for the
// method); shared by the standalone kernel and the persistent batch kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "zm_internal.h"

namespace zmk {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef float float8 __attribute__((ext_vector_type(8)));

constexpr int kWaves = 4;

// The rings of an output block are summed in kChunks contiguous chunks whose
// partial sums are added in chunk order, ((c0 + c1) + c2) + c3, whichever
// waves compute them: one wave running through all chunks (NP = 1), two
// waves (NP = 2: the first keeps c0 + c1, the second c2 and c3 apart) or one
// wave per chunk (NP = kChunks), meeting in LDS.  The result is the same bits
// every way, so a launch can pick the split that suits its size.
constexpr int kChunks = 4;

// First ring of chunk c: the block's K steps (16 rings, or 32 for the 16-bit
// splits) dealt out in contiguous runs.
__device__ __forceinline__ int chunk_edge(int Rp, int step, int c) { return ((Rp / step) * c / kChunks) * step; }

// LDS one output block needs when its chunks are split over waves: [chunk][16][64] values.
template <int DT>
constexpr size_t chunk_lds_bytes() {
    return (size_t)kChunks * 16 * 64 * (DT == ZM_F64 ? sizeof(double) : sizeof(float));
}

__device__ __forceinline__ int out_index(int n, int m) { return zm::canon_index(n, m); }


// frame scale for the F16 split: 2^e with max|F| * 2^e in [2^13, 2^14)
__device__ __forceinline__ float f16_frame_scale(float mx) {
    if (!(mx > 0.f)) return 1.f;
    int ex;
    frexpf(mx, &ex);
    return ldexpf(1.f, 14 - ex);
}

struct ProjArgs {
    const zm_item* items;
    int n_units, ncb;
    const void* thi;
    const void* tlo;
    const float* rowscale;
    const void* F;
    const float* fmaxbuf;
    int B, M, Rp, Mtot;
    void* Z;             // contiguous [B][Mtot][2], or null
    void* const* Zptrs;  // per-frame outputs (used when Z is null)
};

template <typename T>
__device__ __forceinline__ T* zbase(const ProjArgs& a, int fr) {
    // the per-frame pointers are read as pointers to global memory, so that
    // the stores through them are global stores rather than flat ones
    using GP = __attribute__((address_space(1))) T*;
    return a.Z ? (T*)a.Z + (size_t)fr * a.Mtot * 2 : (T*)((const GP*)(const void*)a.Zptrs)[fr];
}

// Output block `unit` = (item unit / ncb, column block unit % ncb).  With
// NP = 1 this wave computes the whole block; with NP = kChunks it computes
// chunk `part`, the NP waves of the block run together in one workgroup and
// meet at barriers (a wave with valid == false, a block past the end,
// computes nothing but still reaches them), red is the block's
// chunk_lds_bytes<DT>() of LDS.
template <int DT, int NP>
__device__ __forceinline__ void project_unit(const ProjArgs& a, int unit, int lane, int part, bool valid, void* red) {
    static_assert(NP == 1 || NP == 2 || NP == kChunks, "1, 2 or kChunks waves per block");
    using Acc = typename std::conditional<DT == ZM_F64, doublex4, floatx4>::type;
    using Val = typename std::conditional<DT == ZM_F64, double, float>::type;
    if (!valid) unit = 0;
    const zm_item* __restrict__ items = a.items;
    const void* __restrict__ thi = a.thi;
    const void* __restrict__ tlo = a.tlo;
    const float* __restrict__ rowscale = a.rowscale;
    const void* __restrict__ Fv = a.F;
    const float* __restrict__ fmaxbuf = a.fmaxbuf;
    const int B = a.B, M = a.M, Rp = a.Rp, ncb = a.ncb;
    const int li = lane & 15, lg = lane >> 4;
    const int cb = unit % ncb;
    const zm_item it = items[unit / ncb];
    const int m = it.m;
    const bool two = it.rows > 16;  // wave-uniform

    // the two 16-column sub-tiles: column = 2 * frame + (re|im); a column's
    // rings k sit at boff + (k / 16) * TS + k % 16
    const int nRT = Rp / zm::kRingTile;
    const size_t TS = (size_t)M * 2 * zm::kRingTile;
    int col[2], fr[2];
    size_t boff[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        col[u] = cb * 32 + 16 * u + li;
        fr[u] = col[u] >> 1;
        const int frc = fr[u] < B ? fr[u] : B - 1;  // clamp: loads stay in bounds, results discarded
        boff[u] = ((size_t)frc * nRT * M + m) * 2 * zm::kRingTile + (size_t)(col[u] & 1) * zm::kRingTile;
    }
    // operand rows of the two 16-row sub-tiles (zm::op_index layout): lane li's
    // ring group at ring k starts at aoff[s] + k * 16
    constexpr int kG = (DT == ZM_F64 || DT == ZM_F32) ? 4 : 8;
    size_t aoff[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) aoff[s] = zm::op_index(it.toff + it.row0 + 16 * s, 0, Rp, kG) + (size_t)li * kG;

    // this wave's chunks [c0, c1) and their rings [kb, ke)
    constexpr int STEP = (DT == ZM_F64 || DT == ZM_F32) ? 16 : 32;
    const int c0 = part * (kChunks / NP), c1 = c0 + kChunks / NP;
    const int kb = chunk_edge(Rp, STEP, c0);
    const int ke = valid ? chunk_edge(Rp, STEP, c1) : kb;
    Acc acc[2][2] = {};
    Acc tot[2][2] = {};  // sum of the finished leading chunks, in order (NP = 1; wave 0 of NP = 2)
    Val* rd = (Val*)red;
    // the accumulators hold chunk c: fold them into the running total (NP =
    // 1, and chunks 0 and 1 of NP = 2, whose total then goes to LDS slot 0)
    // or hand them to LDS slot c, and clear them for the next chunk
    auto flush = [&](int c) {
        const bool running = NP == 1 || (NP == 2 && part == 0);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (running) {
                    if (c == 0)
                        tot[s][u] = acc[s][u];
                    else
#pragma unroll
                        for (int v = 0; v < 4; ++v) tot[s][u][v] = tot[s][u][v] + acc[s][u][v];
                    if (NP == 2 && c == 1)
#pragma unroll
                        for (int v = 0; v < 4; ++v) rd[((s * 2 + u) * 4 + v) * 64 + lane] = tot[s][u][v];
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) rd[(c * 16 + (s * 2 + u) * 4 + v) * 64 + lane] = acc[s][u][v];
                }
                acc[s][u] = Acc{};
            }
    };
    // chunk c's rings end at ce(c); a wave with valid == false runs no rings
    auto ce = [&](int c) { return valid ? chunk_edge(Rp, STEP, c + 1) : kb; };

    float fsc[2] = {1.f, 1.f};
    if constexpr (DT == ZM_F64) {
        const double* T = (const double*)thi;
        const double* F = (const double*)Fv;
        int k0 = kb;
#pragma unroll 1
        for (int c = c0; c < c1; flush(c), ++c)
        for (const int kc = ce(c); k0 < kc; k0 += 16) {
            const int kk = k0 + 4 * lg;
            double av[2][4], bv[2][4];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (s == 1 && !two) break;
                const double2 x0 = *(const double2*)(T + aoff[s] + (size_t)kk * 16);
                const double2 x1 = *(const double2*)(T + aoff[s] + (size_t)kk * 16 + 2);
                av[s][0] = x0.x; av[s][1] = x0.y; av[s][2] = x1.x; av[s][3] = x1.y;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const size_t fo = boff[u] + (size_t)(k0 >> 4) * TS + 4 * lg;
                const double2 y0 = *(const double2*)(F + fo);
                const double2 y1 = *(const double2*)(F + fo + 2);
                bv[u][0] = y0.x; bv[u][1] = y0.y; bv[u][2] = y1.x; bv[u][3] = y1.y;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    if (s == 1 && !two) break;
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        acc[s][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][v], bv[u][v], acc[s][u], 0, 0, 0);
                }
        }
    } else if constexpr (DT == ZM_F32) {
        const float* T = (const float*)thi;
        const float* F = (const float*)Fv;
        // operand fragments run two ring steps ahead of the MFMAs
        float4 a1[2] = {}, b1[2] = {}, a2[2] = {}, b2[2] = {};
        // operands addressed by 32-bit byte offsets from a wave-uniform base (the
        // loads then take the base from scalar registers): the table from its
        // start, the spectra from the column block's first frame (the block's
        // 16 frames span far less than 2^32 bytes)
        const char* Tb = (const char*)T;
        const size_t fbase = (size_t)(__builtin_amdgcn_readfirstlane(cb) * 16) * nRT * M * 2 * zm::kRingTile;
        const char* Fb = (const char*)(F + fbase);
        const unsigned ta0 = (unsigned)(aoff[0] * 4), ta1 = (unsigned)(aoff[1] * 4);
        const unsigned fb0 = (unsigned)((boff[0] - fbase) * 4), fb1 = (unsigned)((boff[1] - fbase) * 4);
        auto load = [&](int k0, float4* ar, float4* br) {
            const unsigned ko = (unsigned)(k0 + 4 * lg) * 64u;
            ar[0] = *(const float4*)(Tb + (ta0 + ko));
            ar[1] = two ? *(const float4*)(Tb + (ta1 + ko)) : float4{0.f, 0.f, 0.f, 0.f};
            const unsigned fo = (unsigned)(k0 >> 4) * (unsigned)(TS * 4) + (unsigned)(16 * lg);
            br[0] = *(const float4*)(Fb + (fb0 + fo));
            br[1] = *(const float4*)(Fb + (fb1 + fo));
        };
        if (kb < ke) load(kb, a1, b1);
        if (kb + 16 < ke) load(kb + 16, a2, b2);
        int k0 = kb;
#pragma unroll 1
        for (int c = c0; c < c1; flush(c), ++c)
        for (const int kc = ce(c); k0 < kc; k0 += 16) {
            const float4 ar[2] = {a1[0], a1[1]}, br[2] = {b1[0], b1[1]};
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                a1[u] = a2[u];
                b1[u] = b2[u];
            }
            if (k0 + 32 < ke) load(k0 + 32, a2, b2);
            const float av[2][4] = {{ar[0].x, ar[0].y, ar[0].z, ar[0].w}, {ar[1].x, ar[1].y, ar[1].z, ar[1].w}};
            const float bv[2][4] = {{br[0].x, br[0].y, br[0].z, br[0].w}, {br[1].x, br[1].y, br[1].z, br[1].w}};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    acc[0][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0][v], bv[u][v], acc[0][u], 0, 0, 0);
                if (two) {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        acc[1][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1][v], bv[u][v], acc[1][u], 0, 0, 0);
                }
            }
        }
    } else {
        // split forms: 16-bit hi/lo operands, K step 32 (8 consecutive rings per lane group)
        using H8 = typename std::conditional<DT == ZM_BF16X2, bf16x8, halfx8>::type;
        using H1 = typename std::conditional<DT == ZM_BF16X2, __bf16, _Float16>::type;
        const H1* Th = (const H1*)thi;
        const H1* Tl = (const H1*)tlo;
        const float* F = (const float*)Fv;
        if constexpr (DT == ZM_F16X2) {
#pragma unroll
            for (int u = 0; u < 2; ++u) fsc[u] = f16_frame_scale(fmaxbuf[fr[u] < B ? fr[u] : B - 1]);
        }
        // raw operand fragments of ring step k0 + 32 are loaded while step k0 runs
        H8 nah[2] = {}, nal[2] = {};
        float4 ny[2][2];
        auto load = [&](int k0) {
            const int kk = k0 + 8 * lg;
            nah[0] = *(const H8*)(Th + aoff[0] + (size_t)kk * 16);
            nal[0] = *(const H8*)(Tl + aoff[0] + (size_t)kk * 16);
            if (two) {
                nah[1] = *(const H8*)(Th + aoff[1] + (size_t)kk * 16);
                nal[1] = *(const H8*)(Tl + aoff[1] + (size_t)kk * 16);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const size_t fo = boff[u] + (size_t)((k0 >> 4) + (lg >> 1)) * TS + 8 * (lg & 1);
                ny[u][0] = *(const float4*)(F + fo);
                ny[u][1] = *(const float4*)(F + fo + 4);
            }
        };
        if (kb < ke) load(kb);
        int k0 = kb;
#pragma unroll 1
        for (int c = c0; c < c1; flush(c), ++c)
        for (const int kc = ce(c); k0 < kc; k0 += 32) {
            H8 ah[2], al[2], bh[2], bl[2];
            float4 yy[2][2];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                ah[s2] = nah[s2];
                al[s2] = nal[s2];
                yy[s2][0] = ny[s2][0];
                yy[s2][1] = ny[s2][1];
            }
            if (k0 + 32 < ke) load(k0 + 32);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float4 y0 = yy[u][0], y1 = yy[u][1];
                const float yv[8] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float x = yv[e] * fsc[u];
                    const H1 h = (H1)x;
                    bh[u][e] = h;
                    bl[u][e] = (H1)(x - (float)h);
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if constexpr (DT == ZM_BF16X2) {
                    acc[0][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[0], bh[u], acc[0][u], 0, 0, 0);
                    acc[0][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[0], bl[u], acc[0][u], 0, 0, 0);
                    acc[0][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[0], bh[u], acc[0][u], 0, 0, 0);
                    if (two) {
                        acc[1][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[1], bh[u], acc[1][u], 0, 0, 0);
                        acc[1][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[1], bl[u], acc[1][u], 0, 0, 0);
                        acc[1][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[1], bh[u], acc[1][u], 0, 0, 0);
                    }
                } else {
                    acc[0][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[0], bh[u], acc[0][u], 0, 0, 0);
                    acc[0][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[0], bl[u], acc[0][u], 0, 0, 0);
                    acc[0][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[0], bh[u], acc[0][u], 0, 0, 0);
                    if (two) {
                        acc[1][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[1], bh[u], acc[1][u], 0, 0, 0);
                        acc[1][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[1], bl[u], acc[1][u], 0, 0, 0);
                        acc[1][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[1], bh[u], acc[1][u], 0, 0, 0);
                    }
                }
            }
        }
    }

    // epilogue: element v of accumulator (s, u) is output row row_of(s, v) of column col[u]
    const int kmrows = (M - 1 - m) / 2 + 1;
    auto store = [&](int s, int u, int v, Val val) {
        // FP64 MFMA output rows are lane / 16 + 4 v, the FP32 ones 4 (lane / 16) + v
        const int row = it.row0 + 16 * s + (DT == ZM_F64 ? lg + 4 * v : 4 * lg + v);
        if (valid && (s == 0 || two) && row < kmrows && fr[u] < B) {
            if constexpr (DT == ZM_F16X2) val = val * rowscale[it.toff + row] / fsc[u];
            zbase<Val>(a, fr[u])[(size_t)out_index(m + 2 * row, m) * 2 + (col[u] & 1)] = val;
        }
    };
    if constexpr (NP == 1) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) store(s, u, v, tot[s][u][v]);
    } else {
        __syncthreads();
        // wave p writes vector elements [p, p + 1) x (kChunks / NP) of every
        // accumulator: ((c0 + c1) + c2) + c3, with slot 0 holding c0 + c1
        // already when NP = 2
#pragma unroll
        for (int vv = 0; vv < kChunks / NP; ++vv) {
            const int v = part * (kChunks / NP) + vv;
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int e = (s * 2 + u) * 4 + v;
                    Val sum = rd[(0 * 16 + e) * 64 + lane];
#pragma unroll
                    for (int w = NP == 2 ? 2 : 1; w < kChunks; ++w) sum += rd[(w * 16 + e) * 64 + lane];
                    store(s, u, v, sum);
                }
        }
        __syncthreads();
    }
}

}  // namespace zmk
