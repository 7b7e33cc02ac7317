// Radial projection of eq. (1) on the matrix cores.
//
// For each repetition m the outer (radial) sum of eq. (1) is a small dense
// contraction over rings:
//     Z[n, m, (b, re|im)] = sum_r T[n, m, r] * F[b, m, re|im, r],
// with T[n, m, r] = 2(n+1)/(A eps_m) w_r R_nm(rho_r) resident per plan
// (K_m = (n_max - m)/2 + 1 rows per m block, padded to 16) and F the ring
// spectra written by the resample+FFT kernel, blocked by 16-ring tiles:
// F[(((b * nRT + r / 16) * M + m) * 2 + re|im) * 16 + r % 16].
//
// An output block is (m, 16- or 32-row) x (32 columns); columns are
// (frame, re|im).  Its rings are summed in four fixed chunks whose partial
// sums are added in chunk order, by one wave or by four (one per chunk), with
// the same result.  Each lane streams 16-byte rows of both operands straight
// from memory; since only the pairing of k between the A and B fragments
// matters for a contraction, lane group g of every MFMA takes ring
// k0 + 4 g + v (v = element of the 16-byte vector) for both operands.
//
//   ZM_F32   : v_mfma_f32_16x16x4_f32, FP32 operands and accumulation.
//   ZM_F64   : v_mfma_f64_16x16x4_f64.
//   ZM_BF16X2: v_mfma_f32_16x16x32_bf16 on hi/lo splits, three products
//              (hi*hi + hi*lo + lo*hi), FP32 accumulation.
//   ZM_F16X2 : v_mfma_f32_16x16x32_f16, same three products; T rows carry a
//              power-of-two scale (undone per row) and F a per-frame
//              power-of-two scale derived from the frame's max |F|.
// The epilogue writes Z in canonical (n, m) order, [b][idx][re|im].
#include <hip/hip_runtime.h>

#include <type_traits>

#include "project_body.h"

namespace {

using namespace zmk;

ProjArgs make_proj_args(const zm_plan_s* p, const void* F, const float* fmax, int batch, void* Z, void* const* Zptrs) {
    ProjArgs a;
    a.items = p->d_items;
    a.ncb = (2 * batch + 31) / 32;
    a.n_units = (int)p->items.size() * a.ncb;
    a.thi = p->d_thi;
    a.tlo = p->d_tlo;
    a.rowscale = p->d_rowscale;
    a.F = F;
    a.fmaxbuf = fmax;
    a.B = batch;
    a.M = p->n_max + 1;
    a.Rp = p->Rp;
    a.Mtot = p->num_moments;
    a.Z = Z;
    a.Zptrs = Zptrs;
    return a;
}

// Workgroups are dealt round-robin to the 8 XCDs; renumber them so that each
// XCD runs a contiguous range of units.  Units are ordered by m, so the
// row blocks of one m (which all read the same spectra slice F[., m, ., .])
// then share one L2 and the slice comes from HBM once.
// A workgroup of four waves: with NP = 1 each wave owns one output block and
// runs through its rings; with NP = 2 two waves share a block (chunks 0-1
// and 2-3); with NP = kChunks the four waves share one block, one ring chunk
// each; the partial sums are added in chunk order.  Either way the moments
// are the same bits (see project_unit), so the launch picks the split by
// size.
template <int DT, int NP>
__global__ __launch_bounds__(64 * kWaves) void project_kernel(ProjArgs a, int n_blocks) {
    __shared__ __attribute__((aligned(16))) char red[NP == 1 ? 16 : (kWaves / NP) * chunk_lds_bytes<DT>()];
    const int per_xcd = (int)(gridDim.x / 8);
    const int blk = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (blk >= n_blocks) return;  // whole workgroups only: the waves of a block meet at barriers
    if constexpr (NP == 1) {
        const int unit = blk * kWaves + (threadIdx.x >> 6);
        if (unit < a.n_units) project_unit<DT, 1>(a, unit, threadIdx.x & 63, 0, true, red);
    } else {
        // kWaves / NP blocks per workgroup, NP waves each; a wave of a block
        // past the end computes nothing but still meets the barriers
        const int w = threadIdx.x >> 6, unit = blk * (kWaves / NP) + w / NP;
        project_unit<DT, NP>(a, unit < a.n_units ? unit : 0, threadIdx.x & 63, w % NP, unit < a.n_units,
                             red + (size_t)(w / NP) * chunk_lds_bytes<DT>());
    }
}

static_assert(kWaves == kChunks, "a workgroup of one block holds one wave per chunk");

// Waves per output block by launch size (measured at 4K, N_max 200): four
// below 1,024 blocks (small batches, e.g. 425 blocks at batch 1); one from
// 1,024 (batch 64: 1,700 blocks, which fill the MI355X's 1,024 SIMDs about
// twice); two from 2,048 (batch 128: one wave per block left a tail of
// waves per SIMD, 0.131 against 0.111 ms).
constexpr int kBlocksOneWave = 1024;
constexpr int kBlocksTwoWaves = 2048;

template <int DT>
hipError_t launch_dt(const zm_plan_s* p, const void* F, const float* fmax, int batch, void* Z, void* const* Zptrs,
                     hipStream_t s) {
    ProjArgs a = make_proj_args(p, F, fmax, batch, Z, Zptrs);
    if (a.n_units >= kBlocksTwoWaves) {
        const int blocks = (a.n_units + 1) / 2;
        const int blocks8 = (blocks + 7) / 8 * 8;
        hipLaunchKernelGGL((project_kernel<DT, 2>), dim3(blocks8), dim3(64 * kWaves), 0, s, a, blocks);
    } else if (a.n_units >= kBlocksOneWave) {
        const int blocks = (a.n_units + kWaves - 1) / kWaves;
        const int blocks8 = (blocks + 7) / 8 * 8;
        hipLaunchKernelGGL((project_kernel<DT, 1>), dim3(blocks8), dim3(64 * kWaves), 0, s, a, blocks);
    } else {
        const int blocks = a.n_units;
        const int blocks8 = (blocks + 7) / 8 * 8;
        hipLaunchKernelGGL((project_kernel<DT, kChunks>), dim3(blocks8), dim3(64 * kWaves), 0, s, a, blocks);
    }
    return hipGetLastError();
}

// Non-finite values among each frame's moments: block (x, b) scans values
// [x * kScan, (x + 1) * kScan) of frame b (exponent field all ones: NaN or
// Inf) and adds its count to counts[b], one atomic per wave that found any.
constexpr int kScanThreads = 256, kScanPer = 4, kScan = kScanThreads * kScanPer;

template <typename T>
__global__ __launch_bounds__(kScanThreads) void count_nonfinite_kernel(const T* __restrict__ Z, long long per_frame,
                                                                         int* __restrict__ counts) {
    using U = typename std::conditional<sizeof(T) == 8, unsigned long long, unsigned>::type;
    constexpr U kExp = sizeof(T) == 8 ? 0x7ff0000000000000ull : 0x7f800000u;
    const int b = blockIdx.y;
    const U* z = reinterpret_cast<const U*>(Z) + (size_t)b * per_frame;
    const long long base = (long long)blockIdx.x * kScan + threadIdx.x;
    int bad = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const long long e = base + (long long)i * kScanThreads;
        if (e < per_frame) bad += (z[e] & kExp) == kExp ? 1 : 0;
    }
    // wave sum by butterfly; lane 0 of a wave with a non-zero count adds it
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off, 64);
    if ((threadIdx.x & 63) == 0 && bad != 0) atomicAdd(counts + b, bad);
}

}  // namespace

namespace zm {

hipError_t launch_count_nonfinite(const zm_plan_s* p, const void* Z, int batch, int* counts, hipStream_t s) {
    hipError_t e = launch_zero_u32(reinterpret_cast<unsigned*>(counts), (size_t)batch, s);
    if (e != hipSuccess) return e;
    const long long per_frame = 2ll * zm_num_moments(p->n_max);
    const dim3 grid((unsigned)((per_frame + kScan - 1) / kScan), (unsigned)batch);
    if (p->dtype == ZM_F64)
        hipLaunchKernelGGL(count_nonfinite_kernel<double>, grid, dim3(kScanThreads), 0, s, (const double*)Z,
                           per_frame, counts);
    else
        hipLaunchKernelGGL(count_nonfinite_kernel<float>, grid, dim3(kScanThreads), 0, s, (const float*)Z, per_frame,
                           counts);
    return hipGetLastError();
}

static hipError_t launch_any(const zm_plan_s* p, const void* F, const float* fmax, int batch, void* Z,
                             void* const* Zptrs, hipStream_t s) {
    switch (p->dtype) {
        case ZM_F64: return launch_dt<ZM_F64>(p, F, fmax, batch, Z, Zptrs, s);
        case ZM_F32: return launch_dt<ZM_F32>(p, F, fmax, batch, Z, Zptrs, s);
        case ZM_BF16X2: return launch_dt<ZM_BF16X2>(p, F, fmax, batch, Z, Zptrs, s);
        case ZM_F16X2: return launch_dt<ZM_F16X2>(p, F, fmax, batch, Z, Zptrs, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_project(const zm_plan_s* p, const void* F, const float* fmax, int batch, void* Z, hipStream_t s) {
    return launch_any(p, F, fmax, batch, Z, nullptr, s);
}

hipError_t launch_project_ptrs(const zm_plan_s* p, const void* F, const float* fmax, int batch, void* const* Zptrs,
                               hipStream_t s) {
    return launch_any(p, F, fmax, batch, nullptr, Zptrs, s);
}

}  // namespace zm
