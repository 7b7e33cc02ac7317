// Batched persistent form: frames of different sizes and orders in one
// launch.
//
// The host groups the jobs by plan and builds a device work queue:
//   stage-1 items (frame, ring tile)      -> fused resample + ring FFT,
//   stage-2 items (plan group, 8 blocks)  -> radial projection on MFMA.
// One persistent kernel pops items with atomic counters: stage-1 items from
// eight ranges (one per XCD, taking from the others when its own is empty),
// then stage-2 items; a workgroup claims its next item of its own range
// inside the current tile's body, so the atomic overlaps the tile's first
// loads.  A workgroup counts its finished stage-1 tiles and,
// when it moves on to another group, to stage 2 or to the exit, releases
// them (device-scope release fence) and adds them to the group's counter; a
// stage-2 item waits (acquire) until its group's counter reaches the group's
// tile count.  Every stage-1 item is popped before any stage-2 item, stage-1
// items never wait, and a workgroup releases before it takes a stage-2 item,
// so every wait ends; the wait is bounded anyway and reports an error flag
// if the bound trips.
// Each item runs exactly the code of the standalone kernels, so a frame's
// moments are bit-identical alone and in a batch.
//
// A batch object captures [counter reset kernel + persistent kernel] in a
// HIP graph once and replays it; a small autotuner picks the persistent grid
// size and the item order by timing candidates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fft_body.h"
#include "project_body.h"

namespace {

using namespace zmk;
using zm::fail;
using zm::hip_fail;

constexpr int kBatchThreads = 512;
constexpr int kAList[4] = {512, 1024, 2048, 4096};
constexpr int kA2List[5] = {16, 32, 64, 128, 256};

// variants served by the persistent kernel: FP32 transforms with A >= 512
// (512-thread shape), LDS within the batch kernel's budget
template <int A, int A2>
constexpr bool batch_variant_ok() {
    return A2 * 2 <= A && FftLds<float, A, A2>::bytes <= 80 * 1024;  // two workgroups per CU
}

// A stage-1 item is one round of the FFT body: the standalone kernel's tile
// (P ring pairs of one frame, P the pairs the 512-thread body transforms at
// once).
constexpr int kItemPairs = 1;

template <int AI, int A2I>
constexpr size_t lds_of() {
    if constexpr (batch_variant_ok<kAList[AI], kA2List[A2I]>())
        return FftLds<float, kAList[AI], kA2List[A2I]>::bytes;
    else
        return 0;
}
constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
template <int AI>
constexpr size_t lds_row() {
    return cmax(cmax(cmax(lds_of<AI, 0>(), lds_of<AI, 1>()), cmax(lds_of<AI, 2>(), lds_of<AI, 3>())), lds_of<AI, 4>());
}
constexpr size_t kBatchLds = cmax(cmax(lds_row<0>(), lds_row<1>()), cmax(lds_row<2>(), lds_row<3>()));

// a stage-2 item: kProjUnits projection output blocks, one wave per ring
// chunk of each (the standalone launch forms the same bits with either split)
constexpr int kProjUnits = kBatchThreads / (64 * kChunks);
static_assert(kProjUnits * chunk_lds_bytes<ZM_F32>() <= kBatchLds, "stage-2 partial sums fit the kernel's LDS");

struct BatchJob {
    FftArgs<float> fa;
    int variant;  // AI * 5 + A2I
    int group;
};

struct BatchGroup {
    ProjArgs pa;
    int dtype;
    unsigned tiles_total;
};

struct BatchItem {
    int kind;  // 0: stage-1 (job, tile), 1: stage-2 (group, kProjUnits output blocks)
    int idx;
    int sub;
    int group;  // stage-1: the job's plan group; stage-2: -1
};


// Reads *p with scalar loads: the address is made wave-uniform and the read
// goes through the constant address space (the tables are written by the
// host before the launch and only read by the kernel).
template <class T>
__device__ __forceinline__ T uniform_load(const T* p) {
    using CU = const __attribute__((address_space(4))) unsigned;
    const unsigned long long a = (unsigned long long)p;
    CU* q = (CU*)(((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(a >> 32)) << 32) |
                  (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((unsigned)a));
    static_assert(sizeof(T) % 4 == 0, "");
    T out;
    unsigned* o = reinterpret_cast<unsigned*>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) o[k] = q[k];
    return out;
}

// Reads the pointer field *f (in a table of the kernel's) as a pointer to
// global memory, with a scalar load, and returns it as a generic pointer.
// The compiler's address-space inference then makes the accesses through it
// global loads and stores, as for a kernel argument, instead of flat ones
// (which need a 64-bit address per lane and wait on the LDS counter too).
template <class T>
__device__ __forceinline__ T* global_field(T* const* f) {
    using GP = __attribute__((address_space(1))) T*;
    const unsigned long long a = (unsigned long long)f;
    const __attribute__((address_space(4))) GP* q =
        (const __attribute__((address_space(4))) GP*)(((unsigned long long)__builtin_amdgcn_readfirstlane(
                                                            (unsigned)(a >> 32))
                                                        << 32) |
                                                       (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(
                                                           (unsigned)a));
    return (T*)*q;
}

// LDS of the persistent kernel, shared by all item bodies.
__shared__ __attribute__((aligned(16))) char g_batch_smem[kBatchLds];

// Each item body is a separate (non-inlined) function, so that the register
// pressure of one variant does not add to another's.  It reads its job's
// arguments with scalar loads and marks their pointers as global memory, so
// its code matches the standalone kernel's (which gets both from being a
// kernel); the kernel's occupancy target (4 waves per SIMD, two 512-thread
// workgroups per CU, what the LDS allows anyway) bounds every body's
// registers.
// Claim of the next item of a range, issued before a tile body and read
// after it, so that the atomic's latency hides behind the body (a barrier
// waits for LDS operations only, not for this load).
struct Claim {
    unsigned* head;
    int off, len;
};

// Runs one stage-1 tile; thread 0 claims the next item of `c`'s range on the
// way and returns it (-1 on other threads or when the range is exhausted).
template <int AI, int A2I>
__device__ __attribute__((noinline)) int run_tile(const BatchJob* j, int tile, Claim c) {
    unsigned k = 0xffffffffu;
    if (threadIdx.x == 0) k = atomicAdd(c.head, 1u);
    if constexpr (batch_variant_ok<kAList[AI], kA2List[A2I]>()) {
        FftArgs<float> fa = uniform_load(&j->fa);
        fa.src = global_field(&j->fa.src);
        fa.spx = global_field(&j->fa.spx);
        fa.trig = global_field(&j->fa.trig);
        fa.tw = global_field(&j->fa.tw);
        fa.F = global_field(&j->fa.F);
        fa.fmaxbuf = global_field(&j->fa.fmaxbuf);
        tile = __builtin_amdgcn_readfirstlane(tile);
        polar_fft_tile<float, kAList[AI], kA2List[A2I], 512, kItemPairs>(fa, 0, tile, g_batch_smem);
    }
    return k < (unsigned)c.len ? c.off + (int)k : -1;
}

template <int AI>
__device__ __forceinline__ int run_tile_a2(const BatchJob* j, int a2i, int tile, Claim c) {
    switch (a2i) {
        case 0: return run_tile<AI, 0>(j, tile, c);
        case 1: return run_tile<AI, 1>(j, tile, c);
        case 2: return run_tile<AI, 2>(j, tile, c);
        case 3: return run_tile<AI, 3>(j, tile, c);
        case 4: return run_tile<AI, 4>(j, tile, c);
        default: return -1;
    }
}

__device__ __forceinline__ int run_tile_a(const BatchJob* j, int ai, int a2i, int tile, Claim c) {
    switch (ai) {
        case 0: return run_tile_a2<0>(j, a2i, tile, c);
        case 1: return run_tile_a2<1>(j, a2i, tile, c);
        case 2: return run_tile_a2<2>(j, a2i, tile, c);
        case 3: return run_tile_a2<3>(j, a2i, tile, c);
        default: return -1;
    }
}

template <int DT>
__device__ __attribute__((noinline)) void run_proj(const BatchGroup* g, int unit, int lane, int part, bool valid,
                                                   void* red) {
    ProjArgs pa = uniform_load(&g->pa);
    pa.items = global_field(&g->pa.items);
    pa.thi = global_field(&g->pa.thi);
    pa.tlo = global_field(&g->pa.tlo);
    pa.rowscale = global_field(&g->pa.rowscale);
    pa.F = global_field(&g->pa.F);
    pa.fmaxbuf = global_field(&g->pa.fmaxbuf);
    pa.Z = global_field(&g->pa.Z);
    pa.Zptrs = global_field(&g->pa.Zptrs);
    unit = __builtin_amdgcn_readfirstlane(unit);
    project_unit<DT, kChunks>(pa, unit, lane, part, valid, red);
}

__global__ void batch_reset_kernel(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Queues: stage-1 items sit in kQueues contiguous ranges, one per XCD (a
// range holds whole frames in radial order, so rings that share cache lines
// are gathered in one L2); stage-2 items follow in one range.
constexpr int kQueues = 8;
struct QueueInfo {
    int off[kQueues + 1];  // first item of each stage-1 range, then of stage 2
    int len[kQueues + 1];
};
// ctr[q] = head of range q (q <= kQueues), ctr[kQueues + 1] = released
// stage-1 tiles of all groups, ctr[kCtrGroups + g] = released tiles of group
// g, ctr[kCtrGroups + n_groups] = error flag (a wait that hit its bound)
constexpr int kCtrTotal = kQueues + 1;
constexpr int kCtrGroups = kQueues + 2;

// Next item for a workgroup whose home range is `home` (thread 0 only): its
// own range first (unless `skip_home`: a claim on it already failed), then
// the other stage-1 ranges, then stage 2.  Heads only grow, so stage-2 items
// are taken only after every stage-1 item has been taken, and a workgroup
// waiting in stage 2 holds no stage-1 item.
__device__ __forceinline__ int pop_item(const QueueInfo& q, unsigned* ctr, int home, bool skip_home) {
    unsigned h[kQueues];  // all heads read at once: one round trip, not eight
#pragma unroll
    for (int d = 0; d < kQueues; ++d)
        h[d] = __hip_atomic_load(&ctr[(home + d) % kQueues], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int d = 0; d < kQueues; ++d) {
        const int r = (home + d) % kQueues;
        if ((d > 0 || !skip_home) && h[d] < (unsigned)q.len[r]) {
            const unsigned k = atomicAdd(&ctr[r], 1u);
            if (k < (unsigned)q.len[r]) return q.off[r] + (int)k;
        }
    }
    const unsigned k = atomicAdd(&ctr[kQueues], 1u);
    return k < (unsigned)q.len[kQueues] ? q.off[kQueues] + (int)k : -1;
}

__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(4))) void batch_kernel(const BatchItem* __restrict__ items, QueueInfo q,
                                                              const BatchJob* __restrict__ jobs,
                                                              const BatchGroup* __restrict__ groups, int n_groups,
                                                              unsigned* ctr, unsigned spin_limit) {
    __shared__ int cur;
    const int tid = threadIdx.x;
    // workgroups are dealt round-robin to the XCDs
    const int home = (int)(blockIdx.x % kQueues);
    // Thread 0 holds the next item (claimed during the current one).  Every
    // thread tracks the workgroup's finished tiles that are not yet released
    // (`pend` tiles of group `pend_group`; the same in all threads).  A
    // release writes the XCD's L2 back, which stalls the gathers of every
    // workgroup on that XCD, so it is done once per run of tiles of one
    // group: before a tile of another group, before a stage-2 item (which may
    // wait) and before the exit; the waves wait for their stores only then.
    // No stage-2 item is popped while stage-1 items remain, and a workgroup
    // releases before it runs one, so every wait still ends.
    int next = 0, pend_group = -1;
    unsigned pend = 0;
    // Thread 0 also remembers what its last acquire covered: the group it
    // waited for, or every group when all stage-1 tiles had been released
    // by then.  An acquire invalidates the XCD's L2 (the radial tables that
    // other projection items are reusing included), so it is done only when
    // a stage-2 item's group is not covered yet.
    int acq_group = -1;
    bool acq_all = false;
    // device-scope release of the workgroup's finished tiles (thread 0, after
    // a barrier that every wave reached with its stores completed): writes
    // the L2's dirty lines back; a release fence does not invalidate, so the
    // XCD keeps the frame lines that other workgroups gather from
    auto release = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        atomicAdd(&ctr[kCtrGroups + pend_group], pend);
        atomicAdd(&ctr[kCtrTotal], pend);
        pend = 0;
    };
    const Claim claim{&ctr[home], q.off[home], q.len[home]};
    if (tid == 0) next = pop_item(q, ctr, home, false);
    for (;;) {
        __syncthreads();  // previous item's LDS users are done; `cur` is free
        if (tid == 0) cur = next;
        __syncthreads();
        const int i = __builtin_amdgcn_readfirstlane(cur);  // uniform: scalar loads of the item and its job
        const BatchItem it = i >= 0 ? items[i] : BatchItem{-1, -1, 0, -1};
        if (pend && (it.kind != 0 || it.group != pend_group)) {
            // every wave's stores of the pending tiles have completed before
            // the barrier that precedes thread 0's release
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0) release();
            pend = 0;
        }
        if (i < 0) return;
        if (it.kind == 0) {
            const BatchJob* j = jobs + it.idx;
            const int variant = j->variant;
            const int claimed = run_tile_a(j, variant / 5, variant % 5, it.sub, claim);
            pend_group = it.group;
            ++pend;
            if (tid == 0) next = claimed >= 0 ? claimed : pop_item(q, ctr, home, true);
        } else {
            const BatchGroup* g = groups + it.idx;
            const unsigned need = g->tiles_total;
            if (tid == 0) next = pop_item(q, ctr, home, true);
            if (tid == 0 && !acq_all && it.idx != acq_group) {
                unsigned spins = 0;
                while (__hip_atomic_load(&ctr[kCtrGroups + it.idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       need) {
                    __builtin_amdgcn_s_sleep(8);
                    if (++spins > spin_limit) {
                        atomicOr(&ctr[kCtrGroups + n_groups], 1u);
                        break;
                    }
                }
                // Acquire the group's spectra (and, when every tile has been
                // released, all groups'): invalidates this CU's vector cache
                // and the XCD's L2, which every wave of the workgroup reads
                // through; the barrier below orders their loads after it.
                acq_all = __hip_atomic_load(&ctr[kCtrTotal], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                          (unsigned)q.off[kQueues];
                acq_group = it.idx;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
            // kProjUnits output blocks per item, kChunks waves each (all waves
            // call in: the waves of a block meet at barriers)
            const int slot = tid / (64 * kChunks);
            const int unit = it.sub * kProjUnits + slot;
            const bool valid = unit < g->pa.n_units;
            void* red = g_batch_smem + (size_t)slot * chunk_lds_bytes<ZM_F32>();
            const int part = (tid >> 6) % kChunks;
            switch (g->dtype) {
                case ZM_F32: run_proj<ZM_F32>(g, unit, tid & 63, part, valid, red); break;
                case ZM_BF16X2: run_proj<ZM_BF16X2>(g, unit, tid & 63, part, valid, red); break;
                case ZM_F16X2: run_proj<ZM_F16X2>(g, unit, tid & 63, part, valid, red); break;
                default: break;
            }
        }
    }
}

int a_index(int A) {
    for (int i = 0; i < 4; ++i)
        if (kAList[i] == A) return i;
    return -1;
}
int a2_index(int A2) {
    for (int i = 0; i < 5; ++i)
        if (kA2List[i] == A2) return i;
    return -1;
}

template <int AI, int A2I>
bool host_ok() {
    return batch_variant_ok<kAList[AI], kA2List[A2I]>();
}
bool variant_ok(int ai, int a2i) {
    static const bool tab[4][5] = {
        {host_ok<0, 0>(), host_ok<0, 1>(), host_ok<0, 2>(), host_ok<0, 3>(), host_ok<0, 4>()},
        {host_ok<1, 0>(), host_ok<1, 1>(), host_ok<1, 2>(), host_ok<1, 3>(), host_ok<1, 4>()},
        {host_ok<2, 0>(), host_ok<2, 1>(), host_ok<2, 2>(), host_ok<2, 3>(), host_ok<2, 4>()},
        {host_ok<3, 0>(), host_ok<3, 1>(), host_ok<3, 2>(), host_ok<3, 3>(), host_ok<3, 4>()}};
    return ai >= 0 && a2i >= 0 && tab[ai][a2i];
}
// ring pairs per stage-1 item
int pairs_of(int A) {
    switch (A) {
        case 512: return FftShape<float, 512, 512, kItemPairs>::PAIRS;
        case 1024: return FftShape<float, 1024, 512, kItemPairs>::PAIRS;
        case 2048: return FftShape<float, 2048, 512, kItemPairs>::PAIRS;
        default: return FftShape<float, 4096, 512, kItemPairs>::PAIRS;
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

struct zm_batch_s {
    int device = 0;
    int njobs = 0, ngroups = 0;
    std::vector<zm_plan_t> plans;           // per job
    std::vector<int> job_group, job_slot;   // group and position in the group
    std::vector<std::vector<int>> members;  // jobs of each group
    std::vector<BatchJob> hjobs;
    std::vector<BatchGroup> hgroups;
    std::vector<BatchItem> stage1, stage2;  // natural order
    std::vector<std::vector<void*>> zptrs;  // per group
    std::vector<BatchItem> hitems;          // queue as uploaded (held until the copy has completed)
    std::vector<void*> hzptrs;
    int n_items = 0;
    QueueInfo qinfo{};
    int grid = 0;
    int order = 0;  // 0: cost-descending stage 1, 1: natural
    // 0: the persistent kernel; 1: per plan, the standalone resample + FFT and
    // projection launches (needs each plan's frames at one stride)
    int route = 0;
    bool want_per_plan = false;  // ZM_BATCH_PER_PLAN, or the tuner's choice
    // device memory: one block, laid out by batch_layout
    size_t o_items = 0, o_jobs = 0, o_groups = 0, o_zptr = 0, o_zero = 0;
    std::vector<size_t> foff;  // spectra of each group
    std::vector<size_t> zoff;  // first output slot of each group
    char* d_mem = nullptr;
    bool owns_mem = false;
    size_t d_bytes = 0;
    BatchItem* d_items = nullptr;
    BatchJob* d_jobs = nullptr;
    BatchGroup* d_groups = nullptr;
    void** d_zptrs = nullptr;
    unsigned* d_zero = nullptr;  // counters + F16 max slots (cleared before every run)
    int n_zero = 0;
    hipStream_t stream = nullptr;  // the batch's own stream: uploads, autotuning, capture
    hipEvent_t done = nullptr;     // completion of the last run
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned spin_limit = 1u << 24;
    bool refs_taken = false;       // counted in its plans' batch references
};

namespace {

// Copies the queue (in the current item order), descriptors and output
// pointers to the device, asynchronously on `s`; the host copies stay in the
// batch until the caller has synchronised `s`.
// Orders the queue (current item order, stage 1 split into the per-XCD
// ranges) into b->hitems and the output pointers into b->hzptrs.
void prepare_queue(zm_batch_s* b) {
    std::vector<BatchItem> s1 = b->stage1;
    if (b->order == 0) {
        std::stable_sort(s1.begin(), s1.end(), [&](const BatchItem& x, const BatchItem& y) {
            const zm_plan_s* px = b->plans[x.idx];
            const zm_plan_s* py = b->plans[y.idx];
            return (long)px->A * pairs_of(px->A) > (long)py->A * pairs_of(py->A);
        });
    }
    // split stage 1 into kQueues contiguous ranges of about equal cost (samples per item)
    auto cost = [&](const BatchItem& x) {
        const zm_plan_s* px = b->plans[x.idx];
        return (double)px->A * pairs_of(px->A);
    };
    double total = 0.0;
    for (const BatchItem& x : s1) total += cost(x);
    size_t pos = 0;
    double acc = 0.0;
    for (int r = 0; r < kQueues; ++r) {
        b->qinfo.off[r] = (int)pos;
        const double target = total * (r + 1) / kQueues;
        while (pos < s1.size() && (r == kQueues - 1 || acc + 0.5 * cost(s1[pos]) < target)) acc += cost(s1[pos++]);
        b->qinfo.len[r] = (int)pos - b->qinfo.off[r];
    }
    b->qinfo.off[kQueues] = (int)s1.size();
    b->qinfo.len[kQueues] = (int)b->stage2.size();
    b->hitems.clear();
    b->hitems.insert(b->hitems.end(), s1.begin(), s1.end());
    b->hitems.insert(b->hitems.end(), b->stage2.begin(), b->stage2.end());
    b->n_items = (int)b->hitems.size();
    b->hzptrs.clear();
    for (auto& v : b->zptrs) b->hzptrs.insert(b->hzptrs.end(), v.begin(), v.end());
}

zm_status upload(zm_batch_s* b, hipStream_t s) {
    prepare_queue(b);
    ZM_HIP(hipMemcpyAsync(b->d_items, b->hitems.data(), b->hitems.size() * sizeof(BatchItem), hipMemcpyHostToDevice, s));
    ZM_HIP(hipMemcpyAsync(b->d_jobs, b->hjobs.data(), b->hjobs.size() * sizeof(BatchJob), hipMemcpyHostToDevice, s));
    ZM_HIP(hipMemcpyAsync(b->d_groups, b->hgroups.data(), b->hgroups.size() * sizeof(BatchGroup),
                          hipMemcpyHostToDevice, s));
    ZM_HIP(hipMemcpyAsync(b->d_zptrs, b->hzptrs.data(), b->hzptrs.size() * sizeof(void*), hipMemcpyHostToDevice, s));
    return ZM_OK;
}

zm_status upload_sync(zm_batch_s* b) {
    zm_status st = upload(b, b->stream);
    if (st != ZM_OK) return st;
    ZM_HIP(hipStreamSynchronize(b->stream));
    return ZM_OK;
}

// Elements between consecutive frames of group g when its frames (in slot
// order) sit at one stride of at least H * W floats, else -1.
long long group_stride(const zm_batch_s* b, int g) {
    const std::vector<int>& m = b->members[g];
    const zm_plan_s* p = b->plans[m[0]];
    const long long hw = (long long)p->H * p->W;
    if (m.size() == 1) return hw;
    // addresses compared as integers: the frames may be separate allocations
    auto addr = [&](int k) { return (long long)(uintptr_t)b->hjobs[m[k]].fa.src; };
    const long long d = addr(1) - addr(0);
    if (d <= 0 || d % (long long)sizeof(float) != 0 || d / (long long)sizeof(float) < hw) return -1;
    for (size_t k = 2; k < m.size(); ++k)
        if (addr((int)k) - addr(0) != (long long)k * d) return -1;
    return d / (long long)sizeof(float);
}

bool per_plan_ok(const zm_batch_s* b) {
    for (int g = 0; g < b->ngroups; ++g)
        if (group_stride(b, g) < 0) return false;
    return true;
}

// The per-plan route: counters and FP16 max slots cleared, then for each plan
// the standalone resample + FFT and projection launches over its frames (the
// same kernels as zm_moments, so the same bits), spectra in the batch's memory,
// moments through the batch's output pointers.
hipError_t enqueue_per_plan(zm_batch_s* b, hipStream_t s) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3((b->n_zero + 255) / 256), dim3(256), 0, s, b->d_zero, b->n_zero);
    hipError_t e = hipGetLastError();
    for (int g = 0; g < b->ngroups && e == hipSuccess; ++g) {
        const std::vector<int>& m = b->members[g];
        const zm_plan_s* p = b->plans[m[0]];
        const BatchGroup& G = b->hgroups[g];
        const int n = (int)m.size();
        float* fmax = const_cast<float*>(G.pa.fmaxbuf);
        void* F = b->d_mem + b->foff[g];
        e = zm::launch_polar_fft(p, b->hjobs[m[0]].fa.src, group_stride(b, g), n, F, fmax, 0, s);
        if (e == hipSuccess) e = zm::launch_project_ptrs(p, F, fmax, n, b->d_zptrs + b->zoff[g], s);
    }
    return e;
}

hipError_t enqueue(zm_batch_s* b, hipStream_t s) {
    if (b->route == 1) return enqueue_per_plan(b, s);
    hipLaunchKernelGGL(batch_reset_kernel, dim3((b->n_zero + 255) / 256), dim3(256), 0, s, b->d_zero, b->n_zero);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_kernel, dim3(b->grid), dim3(kBatchThreads), 0, s, b->d_items, b->qinfo, b->d_jobs,
                       b->d_groups, b->ngroups, b->d_zero, b->spin_limit);
    return hipGetLastError();
}

zm_status capture(zm_batch_s* b) {
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    ZM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue(b, b->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess) return hip_fail(e, "batch launch capture");
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    b->graph = g;
    ZM_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return ZM_OK;
}

std::string signature(const zm_batch_s* b) {
    hipDeviceProp_t prop;
    std::string sig;
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) sig = prop.gcnArchName;
    std::vector<std::string> parts;
    for (int i = 0; i < b->njobs; ++i) {
        const zm_plan_s* p = b->plans[i];
        char buf[96];
        std::snprintf(buf, sizeof buf, "%dx%d:n%d:r%d:a%d:t%d", p->H, p->W, p->n_max, p->R, p->A, (int)p->dtype);
        parts.push_back(buf);
    }
    std::sort(parts.begin(), parts.end());
    for (auto& q : parts) sig += "|" + q;
    return sig;
}

// A tuned shape: persistent grid, stage-1 item order, and the route (0:
// persistent kernel, 1: per-plan launches).
struct TunedShape {
    int grid, order, route;
};
std::mutex g_tune_mu;
std::map<std::string, TunedShape> g_tune;  // batch signature -> shape
bool g_tune_loaded = false;

void tune_cache_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("ZM_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[8192];
    while (std::fgets(line, sizeof line, f)) {
        // one entry per line: <grid> <order> <route> <signature> (an entry
        // without the route field is a persistent-kernel shape)
        int grid = 0, order = 0, route = 0, n = 0;
        const int got = std::sscanf(line, "%d %d %d %n", &grid, &order, &route, &n);
        if (got != 3) {
            route = 0;
            if (std::sscanf(line, "%d %d %n", &grid, &order, &n) != 2) continue;
        }
        if (grid > 0 && (order == 0 || order == 1) && (route == 0 || route == 1)) {
            std::string sig(line + n);
            while (!sig.empty() && (sig.back() == '\n' || sig.back() == '\r')) sig.pop_back();
            g_tune[sig] = TunedShape{grid, order, route};
        }
    }
    std::fclose(f);
}

void tune_cache_store(const std::string& sig, const TunedShape& t) {
    g_tune[sig] = t;
    const char* path = std::getenv("ZM_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %d %s\n", t.grid, t.order, t.route, sig.c_str());
    std::fclose(f);
}

// Reads the error flag of the last run, which must have completed; the copy
// runs on `s` and waits for nothing else on the device.
zm_status check_error_flag(zm_batch_s* b, hipStream_t s) {
    unsigned flag = 0;
    ZM_HIP(hipMemcpyAsync(&flag, b->d_zero + kCtrGroups + b->ngroups, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    ZM_HIP(hipStreamSynchronize(s));
    if (flag) return fail(ZM_EDEVICE, "batch kernel: a projection item waited past its bound");
    return ZM_OK;
}

// Times every shape on the batch's own frames (three runs each, the best of
// the last two) and keeps the fastest: persistent grid x item order, and the
// per-plan launches when every plan's frames sit at one stride.  The choice is
// cached per batch signature.  The moments do not depend on the shape.
zm_status autotune(zm_batch_s* b, int cus) {
    const std::string sig = signature(b);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load();
    auto it = g_tune.find(sig);
    if (it != g_tune.end()) {
        b->grid = it->second.grid;
        b->order = it->second.order;
        b->want_per_plan = b->want_per_plan || it->second.route == 1;
        b->route = b->want_per_plan && per_plan_ok(b) ? 1 : 0;
        return upload_sync(b);
    }
    hipEvent_t e0, e1;
    ZM_HIP(hipEventCreate(&e0));
    ZM_HIP(hipEventCreate(&e1));
    auto time_it = [&](float* out) -> zm_status {
        float ms_best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            ZM_HIP(hipEventRecord(e0, b->stream));
            hipError_t e = enqueue(b, b->stream);
            if (e != hipSuccess) return hip_fail(e, "batch launch");
            ZM_HIP(hipEventRecord(e1, b->stream));
            ZM_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            ZM_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) ms_best = std::min(ms_best, ms);
        }
        *out = ms_best;
        return ZM_OK;
    };
    float best = 1e30f;
    TunedShape bt{2 * cus, 0, 0};
    const int grids[3] = {cus, 2 * cus, 4 * cus};
    b->route = 0;
    for (int order = 0; order < 2; ++order) {
        b->order = order;
        zm_status st = upload_sync(b);
        if (st != ZM_OK) return st;
        for (int gi = 0; gi < 3; ++gi) {
            b->grid = grids[gi];
            float ms = 0.f;
            st = time_it(&ms);
            if (st != ZM_OK) return st;
            if (ms < best) {
                best = ms;
                bt = TunedShape{grids[gi], order, 0};
            }
        }
    }
    if (per_plan_ok(b)) {
        b->route = 1;
        float ms = 0.f;
        zm_status st = time_it(&ms);
        if (st != ZM_OK) return st;
        if (ms < best) {
            best = ms;
            bt.route = 1;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->route = 0;
    zm_status st = check_error_flag(b, b->stream);
    if (st != ZM_OK) return st;
    b->grid = bt.grid;
    b->order = bt.order;
    b->want_per_plan = b->want_per_plan || bt.route == 1;
    b->route = b->want_per_plan && per_plan_ok(b) ? 1 : 0;
    tune_cache_store(sig, bt);
    return upload_sync(b);
}

void take_refs(zm_batch_s* b, int delta) {
    for (int g = 0; g < b->ngroups; ++g) zm::add_batch_ref(b->plans[b->members[g][0]], delta);
}

void destroy_batch(zm_batch_s* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    if (b->d_mem && b->owns_mem) (void)hipFree(b->d_mem);
    if (b->refs_taken) take_refs(b, -1);
    delete b;
}

zm_status fill_pointers(zm_batch_s* b, const zm_job* jobs) {
    for (int i = 0; i < b->njobs; ++i) {
        if (!jobs[i].d_image || !jobs[i].d_Z) return fail(ZM_EINVAL, "job with a null frame or output pointer");
        b->hjobs[i].fa.src = (const float*)jobs[i].d_image;
        b->zptrs[b->job_group[i]][b->job_slot[i]] = jobs[i].d_Z;
    }
    return ZM_OK;
}

// Stage-1 items, the jobs' variants and the groups' tile counts (what a
// stage-2 item waits for).
void build_stage1(zm_batch_s* b) {
    b->stage1.clear();
    for (auto& G : b->hgroups) G.tiles_total = 0;
    for (int i = 0; i < b->njobs; ++i) {
        const zm_plan_s* p = b->plans[i];
        BatchJob& j = b->hjobs[i];
        j.variant = a_index(p->A) * 5 + a2_index(p->A2);
        const int tiles = p->Rp / (2 * pairs_of(p->A));
        for (int t = 0; t < tiles; ++t) b->stage1.push_back(BatchItem{0, i, t, j.group});
        b->hgroups[j.group].tiles_total += (unsigned)tiles;
    }
}

// Host side of a batch: checks the jobs, groups them by plan, builds the
// stage-1 and stage-2 items and the descriptors, and lays out the device
// memory (b->d_bytes); no device call.
zm_status batch_layout(zm_batch_s* b, const zm_job* jobs, int njobs) {
    b->njobs = njobs;
    b->device = jobs[0].plan ? jobs[0].plan->device : 0;
    if (const char* sl = std::getenv("ZM_BATCH_SPIN_LIMIT")) {
        // bound on a stage-2 item's wait, in polls; a small value exercises
        // the error path of a dependency that does not complete in time
        char* end = nullptr;
        const unsigned long v = std::strtoul(sl, &end, 10);
        if (end != sl && *end == '\0' && v <= 0xffffffffUL) b->spin_limit = (unsigned)v;
    }
    std::map<zm_plan_t, int> gid;
    for (int i = 0; i < njobs; ++i) {
        zm_plan_t p = jobs[i].plan;
        if (!p) return fail(ZM_EINVAL, "job with a null plan");
        if (p->device != b->device) return fail(ZM_EINVAL, "all plans of a batch must be on one device");
        if (p->dtype == ZM_F64 || p->n_max > zm::kMaxMomentOrder || !variant_ok(a_index(p->A), a2_index(p->A2)))
            return fail(ZM_EUNSUPPORTED, "batch jobs need an FP32-family dtype, n_max <= 255 and 512 <= angles <= 4096");
        if (!gid.count(p)) {
            gid[p] = (int)b->members.size();
            b->members.emplace_back();
        }
        b->plans.push_back(p);
        b->job_group.push_back(gid[p]);
        b->job_slot.push_back((int)b->members[gid[p]].size());
        b->members[gid[p]].push_back(i);
    }
    b->ngroups = (int)b->members.size();
    const auto& members = b->members;
    // device memory: per group [F of its frames]; queue; descriptors; output pointers; counters
    b->foff.assign(b->ngroups, 0);
    size_t fbytes = 0;
    for (int g = 0; g < b->ngroups; ++g) {
        const zm_plan_s* p = b->plans[members[g][0]];
        b->foff[g] = fbytes;
        fbytes += align256((size_t)members[g].size() * (size_t)(p->n_max + 1) * 2 * p->Rp * sizeof(float));
    }
    b->n_zero = kCtrGroups + b->ngroups + 1 + njobs;  // heads, group counters, error flag, F16 max per frame
    size_t n_items_max = 0;
    for (int i = 0; i < njobs; ++i) n_items_max += (size_t)b->plans[i]->Rp / (2 * pairs_of(b->plans[i]->A));
    for (int g = 0; g < b->ngroups; ++g) {
        const zm_plan_s* p = b->plans[members[g][0]];
        const size_t units = p->items.size() * ((2 * members[g].size() + 31) / 32);
        n_items_max += (units + kProjUnits - 1) / kProjUnits;
    }
    b->o_items = align256(fbytes);
    b->o_jobs = b->o_items + align256(n_items_max * sizeof(BatchItem));
    b->o_groups = b->o_jobs + align256((size_t)njobs * sizeof(BatchJob));
    b->o_zptr = b->o_groups + align256((size_t)b->ngroups * sizeof(BatchGroup));
    b->o_zero = b->o_zptr + align256((size_t)njobs * sizeof(void*));
    b->d_bytes = b->o_zero + align256((size_t)b->n_zero * sizeof(unsigned));

    b->hjobs.resize(njobs);
    b->zptrs.resize(b->ngroups);
    b->zoff.assign(b->ngroups, 0);
    size_t zbase = 0;
    for (int g = 0; g < b->ngroups; ++g) {
        b->zptrs[g].assign(members[g].size(), nullptr);
        b->zoff[g] = zbase;
        zbase += members[g].size();
    }
    for (int i = 0; i < njobs; ++i) {
        const zm_plan_s* p = b->plans[i];
        const int g = b->job_group[i];
        BatchJob& j = b->hjobs[i];
        j.fa.src = nullptr;
        j.fa.src_stride = (long long)p->H * p->W;
        j.fa.H = p->H;
        j.fa.W = p->W;
        j.fa.cx = p->cx;
        j.fa.cy = p->cy;
        j.fa.safe_s = std::min(p->cx, p->cy) - 1e-6;
        j.fa.R = p->R;
        j.fa.Rp = p->Rp;
        j.fa.M = p->n_max + 1;
        j.fa.from_polar = 0;
        j.fa.spx = p->d_spx;
        j.fa.trig = p->d_trig;
        j.fa.tw = (const float*)p->d_tw;
        j.fa.F = nullptr;
        j.fa.fmaxbuf = nullptr;
        j.group = g;
    }
    b->hgroups.resize(b->ngroups);
    for (int g = 0; g < b->ngroups; ++g) {
        const zm_plan_s* p = b->plans[members[g][0]];
        const int n = (int)members[g].size();
        BatchGroup& G = b->hgroups[g];
        G.pa.items = p->d_items;
        G.pa.ncb = (2 * n + 31) / 32;
        G.pa.n_units = (int)p->items.size() * G.pa.ncb;
        G.pa.thi = p->d_thi;
        G.pa.tlo = p->d_tlo;
        G.pa.rowscale = p->d_rowscale;
        G.pa.F = nullptr;
        G.pa.fmaxbuf = nullptr;
        G.pa.B = n;
        G.pa.M = p->n_max + 1;
        G.pa.Rp = p->Rp;
        G.pa.Mtot = p->num_moments;
        G.pa.Z = nullptr;
        G.pa.Zptrs = nullptr;
        G.dtype = (int)p->dtype;
        const int blocks = (G.pa.n_units + kProjUnits - 1) / kProjUnits;
        for (int k = 0; k < blocks; ++k) b->stage2.push_back(BatchItem{1, g, k, -1});
    }
    build_stage1(b);
    return fill_pointers(b, jobs);
}

// Places the batch's device memory at `mem` (d_bytes bytes, 256-byte
// aligned) and sets the descriptors' pointers into it.
void batch_bind(zm_batch_s* b, char* mem) {
    b->d_mem = mem;
    b->d_items = (BatchItem*)(mem + b->o_items);
    b->d_jobs = (BatchJob*)(mem + b->o_jobs);
    b->d_groups = (BatchGroup*)(mem + b->o_groups);
    b->d_zptrs = (void**)(mem + b->o_zptr);
    b->d_zero = (unsigned*)(mem + b->o_zero);
    unsigned* fmax0 = b->d_zero + kCtrGroups + 1 + b->ngroups;  // F16 max slots, contiguous per group
    for (int i = 0; i < b->njobs; ++i) {
        const zm_plan_s* p = b->plans[i];
        const int g = b->job_group[i], k = b->job_slot[i];
        BatchJob& j = b->hjobs[i];
        j.fa.F = (float*)(mem + b->foff[g]) + (size_t)k * (p->n_max + 1) * 2 * p->Rp;
        j.fa.fmaxbuf = p->dtype == ZM_F16X2 ? (float*)(fmax0 + b->zoff[g] + k) : nullptr;
    }
    for (int g = 0; g < b->ngroups; ++g) {
        const zm_plan_s* p = b->plans[b->members[g][0]];
        BatchGroup& G = b->hgroups[g];
        G.pa.F = mem + b->foff[g];
        G.pa.fmaxbuf = p->dtype == ZM_F16X2 ? (const float*)(fmax0 + b->zoff[g]) : nullptr;
        G.pa.Zptrs = b->d_zptrs + b->zoff[g];
    }
}

int device_cus(int device) {
    hipDeviceProp_t prop;
    const hipError_t e = hipGetDeviceProperties(&prop, device);
    return (e == hipSuccess && prop.multiProcessorCount > 0) ? prop.multiProcessorCount : 256;
}

}  // namespace

using namespace zm;

extern "C" {

zm_status zm_batch_create(const zm_job* jobs, int njobs, int flags, zm_batch_t* out) {
    if (!jobs || !out || njobs <= 0) return fail(ZM_EINVAL, "need a non-empty job list and an output pointer");
    *out = nullptr;
    if (flags & ~(ZM_BATCH_AUTOTUNE | ZM_BATCH_NO_GRAPH | ZM_BATCH_PER_PLAN))
        return fail(ZM_EINVAL, "unknown batch flags");
    zm_batch_s* b = new zm_batch_s();
    zm_status st = batch_layout(b, jobs, njobs);
    if (st != ZM_OK) {
        destroy_batch(b);
        return st;
    }
    ZM_DEVICE(b->device);
    char* mem = nullptr;
    hipError_t e = hipMalloc((void**)&mem, b->d_bytes);
    if (e != hipSuccess) {
        destroy_batch(b);
        return hip_fail(e, "hipMalloc (batch)");
    }
    b->owns_mem = true;
    batch_bind(b, mem);
    take_refs(b, +1);
    b->refs_taken = true;
    const int cus = device_cus(b->device);
    b->grid = 2 * cus;
    b->order = 0;
    b->want_per_plan = (flags & ZM_BATCH_PER_PLAN) != 0;
    b->route = b->want_per_plan && per_plan_ok(b) ? 1 : 0;
    e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        destroy_batch(b);
        return hip_fail(e, "hipStreamCreate / hipEventCreate");
    }
    st = upload_sync(b);
    if (st == ZM_OK && (flags & ZM_BATCH_AUTOTUNE)) st = autotune(b, cus);
    if (st == ZM_OK && !(flags & ZM_BATCH_NO_GRAPH)) st = capture(b);
    if (st != ZM_OK) {
        destroy_batch(b);
        return st;
    }
    log_msg(kLogInfo, "batch %p: %d jobs, %d queue items, %zu device bytes; %s, grid %d, item order %d%s%s",
            (void*)b, njobs, b->n_items, b->d_bytes, b->route ? "per-plan launches" : "persistent kernel", b->grid,
            b->order, (flags & ZM_BATCH_AUTOTUNE) ? " (tuned)" : "", (flags & ZM_BATCH_NO_GRAPH) ? "" : ", graph captured");
    *out = b;
    return ZM_OK;
}

zm_status zm_batch_update(zm_batch_t b, const zm_job* jobs, int njobs) {
    if (!b || !jobs) return fail(ZM_EINVAL, "null batch or jobs");
    if (njobs != b->njobs) return fail(ZM_EINVAL, "job count differs from the batch");
    for (int i = 0; i < njobs; ++i)
        if (jobs[i].plan != b->plans[i]) return fail(ZM_EINVAL, "jobs must keep their plans and order");
    for (int i = 0; i < njobs; ++i)
        if (!jobs[i].d_image || !jobs[i].d_Z) return fail(ZM_EINVAL, "job with a null frame or output pointer");
    ZM_DEVICE(b->device);
    ZM_HIP(hipEventSynchronize(b->done));  // the descriptors may be in use by the last run
    zm_status st = fill_pointers(b, jobs);
    if (st != ZM_OK) return st;
    st = upload_sync(b);
    if (st != ZM_OK) return st;
    // the per-plan launches take the frame pointers as arguments: capture them
    // again (frames no longer at one stride fall back to the persistent kernel)
    const int route = b->want_per_plan && per_plan_ok(b) ? 1 : 0;
    const bool recapture = b->exec && (route == 1 || b->route == 1);
    b->route = route;
    return recapture ? capture(b) : ZM_OK;
}

zm_status zm_batch_run(zm_batch_t b, zm_stream_t stream) {
    if (!b) return fail(ZM_EINVAL, "null batch");
    ZM_DEVICE(b->device);
    hipStream_t s = (hipStream_t)stream;
    if (b->exec) {
        ZM_HIP(hipGraphLaunch(b->exec, s));
    } else {
        hipError_t e = enqueue(b, s);
        if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
    }
    ZM_HIP(hipEventRecord(b->done, s));
    log_msg(kLogDebug, "zm_batch_run: batch %p, stream %p", (void*)b, stream);
    return ZM_OK;
}

zm_status zm_batch_check(zm_batch_t b) {
    if (!b) return fail(ZM_EINVAL, "null batch");
    ZM_DEVICE(b->device);
    ZM_HIP(hipEventSynchronize(b->done));
    return check_error_flag(b, b->stream);
}

zm_status zm_batch_config(zm_batch_t b, int* grid, int* order, int* n_items, size_t* device_bytes) {
    if (!b) return fail(ZM_EINVAL, "null batch");
    if (grid) *grid = b->route == 1 ? 0 : b->grid;
    if (order) *order = b->order;
    if (n_items) *n_items = b->n_items;
    if (device_bytes) *device_bytes = b->d_bytes;
    return ZM_OK;
}

zm_status zm_batch_destroy(zm_batch_t b) {
    if (!b) return fail(ZM_EINVAL, "null batch");
    zm::DeviceGuard guard(b->device);
    if (b->done) (void)hipEventSynchronize(b->done);
    destroy_batch(b);
    return ZM_OK;
}

zm_status zm_moments_batch(const zm_job* jobs, int njobs, zm_stream_t stream) {
    zm_batch_t b = nullptr;
    zm_status st = zm_batch_create(jobs, njobs, ZM_BATCH_NO_GRAPH, &b);
    if (st != ZM_OK) return st;
    st = zm_batch_run(b, stream);
    if (st == ZM_OK) {
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    if (st == ZM_OK) st = check_error_flag(b, (hipStream_t)stream);
    destroy_batch(b);
    return st;
}

zm_status zm_batch_workspace_size(const zm_job* jobs, int njobs, size_t* bytes) {
    if (!jobs || !bytes || njobs <= 0) return fail(ZM_EINVAL, "need a non-empty job list and an output pointer");
    zm_batch_s b;
    zm_status st = batch_layout(&b, jobs, njobs);
    if (st != ZM_OK) return st;
    *bytes = b.d_bytes;
    return ZM_OK;
}

zm_status zm_moments_batch_ws(const zm_job* jobs, int njobs, void* d_ws, size_t ws_bytes, zm_stream_t stream) {
    if (!jobs || njobs <= 0) return fail(ZM_EINVAL, "need a non-empty job list");
    if (!d_ws) return fail(ZM_EINVAL, "null workspace");
    if (((uintptr_t)d_ws & 255) != 0) return fail(ZM_EINVAL, "workspace must be 256-byte aligned");
    zm_batch_s* b = new zm_batch_s();
    zm_status st = batch_layout(b, jobs, njobs);
    if (st == ZM_OK && ws_bytes < b->d_bytes)
        st = fail(ZM_EINVAL, "workspace too small: need " + std::to_string(b->d_bytes) + " bytes");
    if (st != ZM_OK) {
        destroy_batch(b);
        return st;
    }
    zm::DeviceGuard guard(b->device);
    if (guard.err != hipSuccess) {
        destroy_batch(b);
        return hip_fail(guard.err, "hipSetDevice");
    }
    batch_bind(b, (char*)d_ws);
    take_refs(b, +1);
    b->refs_taken = true;
    b->grid = 2 * device_cus(b->device);
    hipStream_t s = (hipStream_t)stream;
    st = upload(b, s);
    if (st == ZM_OK) {
        hipError_t e = enqueue(b, s);
        if (e != hipSuccess) st = hip_fail(e, "batch kernel launch");
    }
    // the host copies of the queue must outlive the uploads, and the error
    // flag is read after the run: wait for the stream in every case
    hipError_t e = hipStreamSynchronize(s);
    if (st == ZM_OK && e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    if (st == ZM_OK) st = check_error_flag(b, s);
    destroy_batch(b);
    return st;
}

// Staging buffer of the asynchronous one-shot: a header, then an image of
// the device block's [o_items, o_zero) range (queue, descriptors, output
// pointers) copied to the device in one transfer.
namespace {
constexpr unsigned kStageMagic = 0x7a6d5354u;  // "zmST"
constexpr size_t kStageHeader = 256;
struct StageHeader {
    unsigned magic;
    unsigned flag;  // the run's error flag, copied back at the end of the enqueued work
};
}  // namespace

zm_status zm_batch_stage_size(const zm_job* jobs, int njobs, size_t* bytes) {
    if (!jobs || !bytes || njobs <= 0) return fail(ZM_EINVAL, "need a non-empty job list and an output pointer");
    zm_batch_s b;
    zm_status st = batch_layout(&b, jobs, njobs);
    if (st != ZM_OK) return st;
    *bytes = kStageHeader + (b.o_zero - b.o_items);
    return ZM_OK;
}

zm_status zm_moments_batch_async(const zm_job* jobs, int njobs, void* d_ws, size_t ws_bytes, void* h_stage,
                                 size_t stage_bytes, zm_stream_t stream) {
    if (!jobs || njobs <= 0) return fail(ZM_EINVAL, "need a non-empty job list");
    if (!d_ws || !h_stage) return fail(ZM_EINVAL, "null workspace or staging buffer");
    if (((uintptr_t)d_ws & 255) != 0) return fail(ZM_EINVAL, "workspace must be 256-byte aligned");
    if (((uintptr_t)h_stage & 15) != 0) return fail(ZM_EINVAL, "staging buffer must be 16-byte aligned");
    zm_batch_s* b = new zm_batch_s();
    zm_status st = batch_layout(b, jobs, njobs);
    if (st == ZM_OK && ws_bytes < b->d_bytes)
        st = fail(ZM_EINVAL, "workspace too small: need " + std::to_string(b->d_bytes) + " bytes");
    const size_t need = kStageHeader + (b->o_zero - b->o_items);
    if (st == ZM_OK && stage_bytes < need)
        st = fail(ZM_EINVAL, "staging buffer too small: need " + std::to_string(need) + " bytes");
    if (st != ZM_OK) {
        destroy_batch(b);
        return st;
    }
    zm::DeviceGuard guard(b->device);
    if (guard.err != hipSuccess) {
        destroy_batch(b);
        return hip_fail(guard.err, "hipSetDevice");
    }
    batch_bind(b, (char*)d_ws);
    b->grid = 2 * device_cus(b->device);
    prepare_queue(b);
    char* img = (char*)h_stage + kStageHeader;  // mirrors d_ws + o_items
    std::memcpy(img, b->hitems.data(), b->hitems.size() * sizeof(BatchItem));
    std::memcpy(img + (b->o_jobs - b->o_items), b->hjobs.data(), b->hjobs.size() * sizeof(BatchJob));
    std::memcpy(img + (b->o_groups - b->o_items), b->hgroups.data(), b->hgroups.size() * sizeof(BatchGroup));
    std::memcpy(img + (b->o_zptr - b->o_items), b->hzptrs.data(), b->hzptrs.size() * sizeof(void*));
    StageHeader hdr{kStageMagic, 0u};
    std::memcpy(h_stage, &hdr, sizeof hdr);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(b->d_mem + b->o_items, img, b->o_zero - b->o_items, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = enqueue(b, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync((char*)h_stage + offsetof(StageHeader, flag), b->d_zero + kCtrGroups + b->ngroups,
                           sizeof(unsigned), hipMemcpyDeviceToHost, s);
    // the plans record the work's completion on `stream` (zm_destroy waits for it)
    for (int g = 0; e == hipSuccess && st == ZM_OK && g < b->ngroups; ++g)
        st = note_call(b->plans[b->members[g][0]], s);
    destroy_batch(b);
    if (e != hipSuccess) return hip_fail(e, "batch upload / launch");
    if (st == ZM_OK) log_msg(kLogDebug, "zm_moments_batch_async: %d jobs, stream %p", njobs, stream);
    return st;
}

zm_status zm_batch_stage_status(const void* h_stage) {
    if (!h_stage) return fail(ZM_EINVAL, "null staging buffer");
    StageHeader hdr;
    std::memcpy(&hdr, h_stage, sizeof hdr);
    if (hdr.magic != kStageMagic) return fail(ZM_EINVAL, "not a staging buffer of zm_moments_batch_async");
    if (hdr.flag) return fail(ZM_EDEVICE, "batch kernel: a projection item waited past its bound");
    return ZM_OK;
}

}  // extern "C"
