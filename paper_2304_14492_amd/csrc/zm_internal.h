// Internal declarations shared by the libzm translation units (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "zm.h"

namespace zm {

// Diagnostics on stderr, chosen by the environment variable ZM_LOG (read
// once): 0 or unset = none, 1 = every failure, 2 = also plan and batch
// set-up (sizes, resident memory, tuned shapes), 3 = also every call that
// enqueues device work.  One line per message, "zm: <level>: <text>".
enum { kLogError = 1, kLogInfo = 2, kLogDebug = 3 };
int log_level();
void log_msg(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// Error detail for zm_last_error (thread-local).
void set_error(const std::string& msg);
zm_status fail(zm_status s, const std::string& msg);
zm_status hip_fail(hipError_t e, const char* what);

#define ZM_HIP(call)                                     \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return zm::hip_fail(e_, #call); \
    } while (0)

// Makes `dev` the current HIP device for the scope and restores the
// caller's device on exit (entry points run on their plan's device without
// changing the caller's state).
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0 && err == hipSuccess) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard&) = delete;
    DeviceGuard& operator=(const DeviceGuard&) = delete;
};

#define ZM_DEVICE(dev)                                             \
    zm::DeviceGuard zm_device_guard_(dev);                         \
    if (zm_device_guard_.err != hipSuccess) return zm::hip_fail(zm_device_guard_.err, "hipSetDevice")

// Largest order the moment kernels serve (the pruned FFT keeps bins
// 0..n_max inside one sub-transform of at most 256 points).
constexpr int kMaxMomentOrder = 255;
constexpr int kMaxTableOrder = 500;
constexpr int kMaxAngles = 4096;
constexpr int kMinAngles = 32;
constexpr int kMaxRings = 4096;
constexpr int kRingTile = 16;   // rings per resample+FFT workgroup
constexpr int kRingPad = 32;    // rings padded to a multiple of this (projection K step)
constexpr int kRowTile = 16;    // projection rows per MFMA tile (per m block)
constexpr int kErrParts = 6;    // partial sums per block of the reconstruction-error reduction
constexpr int kErrOut = 7;      // doubles per frame returned by zm_recon_error

// Position of entry (row, ring r) in the projection operand table.  Rows come
// in blocks of kRowTile (one MFMA row tile); inside a block the rings come in
// groups of g (the consecutive rings one lane reads for one MFMA fragment: 4
// for FP32/FP64, 8 for the 16-bit splits), and a group holds its g rings for
// each of the block's 16 rows in turn.  So the 16 lanes that read one
// fragment read 16 * g contiguous entries, and each group of 4 lanes one
// 64-byte run (the texture path coalesces within groups of 4 lanes).
__host__ __device__ inline size_t op_index(int row, int r, int Rp, int g) {
    return ((size_t)(row / kRowTile) * Rp + (size_t)(r / g) * g) * kRowTile + (size_t)(row % kRowTile) * g + r % g;
}

// Canonical position of (n, m) (n ascending, then m ascending, m = n mod 2 .. n step 2).
__host__ __device__ inline int canon_index(int n, int m) {
    int p = n >> 1;
    int off = (n & 1) ? (p + 1) * (p + 1) : p * (p + 1);
    return off + (m >> 1);
}

}  // namespace zm

// One projection work item: the rows [row0, row0 + rows) of the m block.
struct zm_item {
    int m;
    int row0;   // first row (n = m + 2 * row) inside the block
    int rows;   // 16 or 32
    int toff;   // first table row of the block in the operand table
};

struct zm_plan_s {
    int n_max, H, W, D, R, A, Rp, M, num_moments;
    int A2;         // pruned sub-transform length (16 * Q, >= n_max + 1)
    int NK;         // DFT length of the radial-table relation
    zm_dtype dtype;
    int neumann;
    zm_ring_rule rule;
    int device;
    double cx, cy, rpx;

    std::vector<double> rho, w;          // ring nodes and weights (host)
    std::vector<int> blk_rows;           // K_m per m
    std::vector<int> blk_toff;           // first operand-table row of each m block
    int table_rows;                      // operand-table rows incl. padding
    std::vector<zm_item> items;          // projection work items

    // device memory owned by the plan
    double* d_spx = nullptr;             // rho_r * D/2 (pixels), R
    double* d_trig = nullptr;            // cos/sin(2 pi a / A), [A][2]
    void* d_tw = nullptr;                // FFT twiddles exp(-2 pi i j / A) as (cos, sin), [A][2]
    double* d_table = nullptr;           // R_nm(rho_r), [num_moments][R], FP64 (eq. (7))
    double* d_jac = nullptr;             // per moment (alpha, beta, gamma) of the pixel-centre recurrence
    void* d_thi = nullptr;               // projection operand (or its hi part)
    void* d_tlo = nullptr;               // lo part (split dtypes)
    float* d_rowscale = nullptr;         // per operand row: factor undoing the F16 row scaling
    zm_item* d_items = nullptr;
    int* d_rowmap = nullptr;             // operand row -> canonical idx (-1 for padding)
    // staged resample + FFT (frame pixels through LDS): workgroup size, 0 when
    // the plan uses the direct gather; per (round, sector) staging windows and
    // their row entries, laid out at plan time
    int stage_nthr = 0;
    void* d_stage_win = nullptr;
    int* d_stage_rows = nullptr;
    size_t resident = 0;

    // What zm_destroy checks before freeing (guarded by mu): the completion
    // event of the last call enqueued on each stream, and the number of
    // batch objects built on the plan.
    std::mutex mu;
    std::vector<std::pair<hipStream_t, hipEvent_t>> done;
    int batch_refs = 0;
};

namespace zm {
// Records on `s` the completion of the work just enqueued on plan p (not
// while `s` is being captured into a graph).  Without may_create it only
// reuses one of the plan's events (one is made with the plan), so the call
// allocates nothing; if every event is still pending it records nothing.
zm_status note_call(zm_plan_s* p, hipStream_t s, bool may_create = true);
// Adds `delta` to the plan's count of batch objects built on it.
void add_batch_ref(zm_plan_s* p, int delta);

// Kernels launchers (each returns hipSuccess or the launch error).
hipError_t launch_zrp_table(const zm_plan_s* p, const double* d_rho, const double* d_ck, hipStream_t s);
hipError_t launch_fold(const zm_plan_s* p, const double* d_w, hipStream_t s);
hipError_t launch_polar_fft(const zm_plan_s* p, const void* img, long long stride, int batch, void* F,
                            float* fmax, int from_polar, hipStream_t s);
hipError_t launch_project(const zm_plan_s* p, const void* F, const float* fmax, int batch, void* Z,
                          hipStream_t s);
// As launch_project with frame b's moments written to Zptrs[b] (a device
// array of batch output pointers).
hipError_t launch_project_ptrs(const zm_plan_s* p, const void* F, const float* fmax, int batch, void* const* Zptrs,
                               hipStream_t s);
hipError_t launch_zero_u32(unsigned* p, size_t n, hipStream_t s);
bool resample_supported(int A);
hipError_t launch_resample(const zm_plan_s* p, const void* img, long long stride, int batch, void* P, hipStream_t s);
hipError_t launch_count_nonfinite(const zm_plan_s* p, const void* Z, int batch, int* counts, hipStream_t s);
hipError_t launch_recon_polar(const zm_plan_s* p, const void* Z, int batch, void* out, int one_sided, hipStream_t s);
hipError_t launch_recon_cart(const zm_plan_s* p, const void* Z, int batch, void* out, int one_sided, hipStream_t s);
size_t recon_reduce_blocks(const zm_plan_s* p);
hipError_t launch_recon_error(const zm_plan_s* p, const void* f, const void* g, int batch, double* part,
                              double* out, hipStream_t s);
hipError_t launch_minmax(const zm_plan_s* p, const void* f, void* g, int batch, double* part, double* mm,
                         hipStream_t s);
hipError_t launch_embed(const void* src, int n_rows, int n_cols, long long src_stride, void* dst, int size, int off_r,
                        int off_c, int batch, int is_double, hipStream_t s);
}  // namespace zm
