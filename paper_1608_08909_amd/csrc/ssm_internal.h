// Internal declarations shared by the libssm HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ssm.h"

// Device state behind an ssm_terms handle.
struct ssm_terms {
    int device = 0;
    void* arena = nullptr;  // one allocation holding every fixed-size buffer below
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
    int32_t* stopw = nullptr;   // [4] sweep loop: {stop test fired, sweeps run}
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
    // Node order of the FP32 sweep (all null when off): nodes sorted by
    // (region, delta, id), so that a wavefront's nodes and their neighbours
    // lie close in memory.  The sweep runs on a renumbered copy of the graph
    // (every row keeps its neighbour order) and of its per-node data; each
    // node's arithmetic is unchanged.  The heavy-row lists above then hold
    // new ids.
    int32_t* perm = nullptr;    // [n] new id -> node
    int32_t* inv = nullptr;     // [n] node -> new id
    int32_t* prp = nullptr;     // [n + 1] renumbered CSR
    int32_t* pci = nullptr;     // [nnz]
    void* pdpk = nullptr;       // packed distances, new order
    float* pden32 = nullptr;    // [n]
    int32_t* pprank = nullptr;  // [n]
    int32_t* ppiv = nullptr;    // [kpad] the pivots' new ids
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
void release_cached_scratch();
// Launch-variant override set by ssm_set_variant, or `unset` when none is.
int variant(const char* name, int unset = 0);

// ---- BFS / regions (bfs.hip)
ssm_status mssp(const ssm_csr* g, int32_t k, const int32_t* pivots, int32_t* dist,
                int32_t* dmax_out_host, hipStream_t s);
ssm_status select_pivots(const ssm_csr* g, int32_t k, int32_t first, int32_t* pivots,
                         hipStream_t s);
// Ids of the nodes with degree > kHeavyDegree, ascending; *heavy holds
// max(count, 1) ints from the scratch cache (salloc), which the caller
// returns with sfree once its stream is idle.  Synchronizes.
ssm_status heavy_list(const ssm_csr* g, int** heavy, int32_t* count, hipStream_t s);

// k-means sp refinement of max/min pivots (kmeans.hip).
ssm_status kmeans_pivots(int32_t n, int32_t k, const int32_t* pivots, const int32_t* dist, int32_t max_iters,
                         int32_t* new_pivots, int32_t* assign, int32_t* iters_host, hipStream_t s);

// Heavy list, its arc segments and the FP32 sweep's scratch for them.
ssm_status heavy_segments(const ssm_csr* g, ssm_terms* t, hipStream_t s);
// FP32 sweep order (when t->perm is allocated) and the heavy-row lists.
ssm_status sweep_order(const ssm_csr* g, ssm_terms* t, const int32_t* delta, const int32_t* region,
                       hipStream_t s);
int sweep_order_mode();  // 0 off, 1 when it pays (build_terms decides), 2 always
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

// ---- layout pool (pool.hip): many small graphs per launch
//
// Device descriptor of one pool graph.  Every graph keeps its own CSR with
// local ids; the batched kernels map a block (or a wave) to a graph through
// an array of these.
constexpr int kPoolMaxN = 65536;  // LDS holds a 2-byte delta per node in the regions stage
constexpr int kPoolMaxK = 256;    // pivot coordinates staged per wave; Gram and eigen step in registers
constexpr int kPoolEllW = 16;     // padded adjacency width
constexpr int kPoolGramChunk = 2048;

struct PoolGraph {
    int n, nnz, k, kpad;   // kpad: k rounded up to 8 (uint16 words)
    int first, W, L, iters;  // max/min start; table row length dmax + 1; delta_max + 1; sweeps in this call
    int parity, ntiles, nchunks, hist;  // FP32 buffer holding the current iterate; Gram tiles, Gram node
                                        // chunks; 1: the FP32 sweep stages Hf and invd in LDS
    const int* rp;          // [n + 1] local arc offsets
    const int* ci;          // [nnz] local ids
    int* ell;               // [n][kPoolEllW] (preparation)
    int* pivots;            // [kpad], padding repeats pivots[0]
    int* dist;              // [k][n] (preparation)
    uint4* dpk;             // [kpad / 8][n] packed uint16 distances
    int* delta;             // [n]
    int* region;            // [n]
    int* H;                 // [k][L] cumulative region histograms (room for k W)
    double* w64;            // [kpad][W]
    float2* wt2;            // [kpad][W]: (w', w' d) in FP32
    float* Hf;              // [kpad][L]: H as float (exact below 2^24), zero rows past k
    float2* invd;           // [W]: (1/d^2, 1/d) for d >= 2, zero below
    double* den64;          // [n]
    float* den32;           // [n]
    double2* x64[2];        // FP64 iterates (PivotMDS, warm-up sweeps)
    float2* x32[2];         // FP32 iterates
    int* m;                 // [n] max/min scratch
    int* gq;                // [3 n] max/min frontier overflow
    long long* colsum;      // [k]
    double* mu;             // [k]
    double* nu;             // [n]
    double* stats;          // [4]
    double* M;              // [k][k]
    double* eig;            // [2 k + 2]
    double* gpart;          // [nchunks][ntiles][256] Gram partial tiles
    int* info;              // [8]: disconnected, dmax, delta_max, zero edge length, eigen steps, invalid
                            // CSR, stop test fired, sweeps run when it fired
    double tol;             // stop test of the FP32 sweeps (0: a fixed sweep count)
    int done0;              // sweeps run before this sweep call
};

// Stages (bfs.hip): fill the max/min scratch and the padded adjacency; one
// max/min selection per graph (one workgroup each); the k BFS per graph as
// (graph, rank) items over a persistent grid with gq_stride ints of overflow
// queue per block.
hipError_t pool_prep_init(const PoolGraph* gs, int count, int nmax, hipStream_t s);
hipError_t pool_select(const PoolGraph* gs, int count, int nmax, hipStream_t s);
int pool_bfs_blocks(int nitems);
hipError_t pool_bfs(const PoolGraph* gs, const int2* items, int nitems, int* gq, long long gq_stride, int blocks,
                    hipStream_t s);
// Stages (pmds.hip): centring statistics, Gram partial tiles as
// (graph, node chunk, tile group) items, their reduction, the eigen step and
// the projection + rescale into x64[0].  tiles lists the 16 x 16 tiles of the
// upper triangle column by column, so a graph with T tile columns uses the
// first T (T + 1) / 2.
hipError_t pool_pivotmds(const PoolGraph* gs, int count, const int4* gram_items, int ngram, const int2* tiles,
                         int kp_max, int k_max, hipStream_t s);

// ---- graphs with edge lengths (wgraph.hip; PivotMDS in pmds.hip)
ssm_status pivotmds_w(const ssm_csr* g, const double* len, int k, const double* dist, ssm_prec p, void* x,
                      hipStream_t s);
ssm_status select_pivots_w(const ssm_csr* g, const double* len, int32_t k, int32_t first, int32_t* pivots,
                           hipStream_t s);
ssm_status sssp_rows(const ssm_csr* g, const double* len, int32_t k, const int32_t* pivots, double* dist,
                     hipStream_t s);

// ---- quality measures (quality.hip)
ssm_status procrustes(int32_t n, int32_t px, const void* x, int32_t py, const void* y, double* out_host,
                      hipStream_t s);
ssm_status procrustes_noalloc(int32_t n, int32_t px, const void* x, int32_t py, const void* y, double* out_host,
                              hipStream_t s);

// Deterministic FP64 sum of `count` partials on the device into out (device).
void launch_sum_partials(const double* partials, int count, double* out, hipStream_t s);

int num_cus();

}  // namespace ssm
