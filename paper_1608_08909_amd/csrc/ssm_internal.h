// Internal declarations shared by the libssm HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ssm.h"

// Device state behind an ssm_terms handle.
struct ssm_terms {
    int device = 0;
    int32_t n = 0, k = 0, nnz = 0;
    int32_t kpad = 0;       // k rounded up to a multiple of vec
    int32_t dmax = 0;       // max hop distance in the table
    int32_t delta_max = 0;  // max distance to the nearest pivot
    int32_t dbytes = 0;     // 1 (dmax <= 255) or 2 bytes per packed distance
    int32_t vec = 0;        // packed distances per 16-byte word (16 or 8)
    int32_t W = 0;          // weight table row length = dmax + 1
    int32_t* pivots = nullptr;  // [kpad], padding repeats pivots[0]
    int32_t* H = nullptr;       // [k][delta_max+1] cumulative region histograms
    double* wtab64 = nullptr;   // [kpad][W], zero rows for padding
    float* wtab32 = nullptr;    // [kpad][W]
    float2* wt2 = nullptr;      // [kpad][W] FP32 (w', w' d) for the FP32 sweep
    float* Hf = nullptr;        // [kpad][delta_max+1] H as float, zero rows for padding
    float2* invd = nullptr;     // [W] (1/d^2, 1/d) for d >= 2, zero below
    int32_t* prank = nullptr;   // [n] rank of the pivot at node i, -1 for other nodes
    float2* pc = nullptr;       // [2][kpad] FP32 sweep: pivot coordinates of the current and next iterate
    double* den64 = nullptr;    // [n]
    float* den32 = nullptr;     // [n]
    void* dpk = nullptr;        // [kpad/vec][n][vec] packed distances (uint8 or uint16)
    void* xtmp = nullptr;       // [n][2] doubles: second buffer of the Jacobi sweeps
    double* red = nullptr;      // reduction scratch, red_len doubles
    int32_t red_len = 0;
    double* eig = nullptr;      // [2k + 2] V (k x 2) then lambda (2)
    double* gram = nullptr;     // [k][k] C^T C of the last PivotMDS
    int32_t* eig_iters = nullptr;  // [1]
    int32_t nheavy = 0;            // nodes whose degree exceeds kHeavyDegree
    int32_t* heavy = nullptr;      // [nheavy] their ids, ascending
    int32_t nseg = 0;              // segments of kHeavySeg arcs over the heavy rows
    int32_t* seg_start = nullptr;  // [nheavy + 1] first segment of each heavy row
    int32_t* seg_owner = nullptr;  // [nseg] heavy row of each segment
    int2* seg_range = nullptr;     // [n] at a heavy node's id: its segments [x, y)
    float2* seg_sum = nullptr;     // [nseg] FP32 sweep scratch: neighbour displacement sum per segment
};

namespace ssm {

// Nodes with more neighbours than this get their neighbour terms summed by
// whole wavefronts in the FP32 sweep, one per segment of kHeavySeg arcs.
constexpr int kHeavyDegree = 64;
constexpr int kHeavySeg = 512;

// Thread-local error reporting.
ssm_status fail(ssm_status st, const std::string& msg);
ssm_status hip_fail(hipError_t e, const char* what);

#define SSM_HIP(call)                                                   \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return ::ssm::hip_fail(e_, #call);        \
    } while (0)

inline int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }

// Validation of ABI arguments that can be checked on the host.
ssm_status check_csr(const ssm_csr* g);

// Device scratch: allocation helper that reports SSM_E_NOMEM.
ssm_status dalloc(void** p, size_t bytes);

// Scratch for the duration of one call: salloc may hand out a cached buffer
// (contents undefined); sfree returns it to the cache.  Release only after
// the stream that used the buffer has been synchronized.
ssm_status salloc(void** p, size_t bytes);
void sfree(void* p);

// ---- BFS / regions (bfs.hip)
ssm_status mssp(const ssm_csr* g, int32_t k, const int32_t* pivots, int32_t* dist,
                int32_t* dmax_out_host, hipStream_t s);
ssm_status select_pivots(const ssm_csr* g, int32_t k, int32_t first, int32_t* pivots,
                         hipStream_t s);
// Ids of the nodes with degree > kHeavyDegree, ascending; *heavy is a new
// device allocation of max(count, 1) ints owned by the caller.  Synchronizes.
ssm_status heavy_list(const ssm_csr* g, int** heavy, int32_t* count, hipStream_t s);

// k-means sp refinement of max/min pivots (kmeans.hip).
ssm_status kmeans_pivots(int32_t n, int32_t k, const int32_t* pivots, const int32_t* dist, int32_t max_iters,
                         int32_t* new_pivots, int32_t* assign, int32_t* iters_host, hipStream_t s);

// Heavy list, its arc segments and the FP32 sweep's scratch for them.
ssm_status heavy_segments(const ssm_csr* g, ssm_terms* t, hipStream_t s);
ssm_status regions(int32_t n, int32_t k, const int32_t* dist, int32_t* delta, int32_t* region,
                   hipStream_t s);

// ---- terms (terms.hip)
ssm_status build_terms(const ssm_csr* g, int32_t k, const int32_t* pivots, const int32_t* dist,
                       const int32_t* delta, const int32_t* region, ssm_terms** out,
                       hipStream_t s);

// ---- PivotMDS (pmds.hip)
ssm_status pivotmds(const ssm_csr* g, ssm_terms* t, ssm_prec p, void* x, hipStream_t s);

// ---- sweeps and stress (sweep.hip)
ssm_status majorize(const ssm_csr* g, ssm_terms* t, ssm_prec p, void* x, int32_t iters,
                    double tol, int32_t* iters_done_host, hipStream_t s);
ssm_status majorize_mixed(const ssm_csr* g, ssm_terms* t, double* x64, float* x32, int32_t iters, int32_t warm,
                          hipStream_t s);
ssm_status stress_sparse(const ssm_csr* g, ssm_terms* t, ssm_prec p, const void* x,
                         double* out_host, hipStream_t s);
ssm_status stress_full(const ssm_csr* g, ssm_prec p, const void* x, double* out_host,
                       hipStream_t s);

// Deterministic FP64 sum of `count` partials on the device into out (device).
void launch_sum_partials(const double* partials, int count, double* out, hipStream_t s);

int num_cus();

}  // namespace ssm
