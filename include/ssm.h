/*
 * ssm.h - C ABI of libssm, the MI355X (gfx950) implementation of the hot path
 * of the sparse stress model (Ortmann, Klimenta, Brandes, "A Sparse Stress
 * Model"): max/min pivot sampling, the pivots' BFS distances, the regions
 * R(p), the adapted weights w'_ip, the PivotMDS start layout and the
 * iterative localized majorization of Eq. 5.
 *
 * Conventions for every call:
 *   - Pointers named *_host are host memory; every other pointer is device
 *     memory on the current HIP device.  The caller owns every buffer except
 *     an ssm_terms handle, which the library owns until ssm_terms_free.
 *   - The graph is a simple undirected graph in symmetric CSR form (Section 1
 *     of the paper): int32 row_ptr[n+1], int32 col_idx[nnz], nnz = 2m, no
 *     self-loops, no duplicate arcs, every arc (u,v) matched by (v,u); edge
 *     lengths are 1 (unweighted).  The method needs a connected graph (the
 *     paper keeps the largest component, Section 4 "Data").  Rows need not be
 *     sorted; the CSR order is the order in which neighbour terms are summed.
 *   - Work is enqueued on `stream`.  A call that returns a value to the host
 *     (a status found on the device, a stress value, an iteration count)
 *     synchronizes that stream before it returns.
 *   - Host-detectable argument errors return before anything is enqueued and
 *     write nothing.  On any status other than SSM_OK, ssm_last_error()
 *     returns a message for the calling thread.
 *   - Layouts x are n x 2 interleaved (x_i^1, x_i^2), of type double for
 *     SSM_FP64 and float for SSM_FP32.
 *   - The distance table dist is k x n int32, pivot-major: row t holds the
 *     hop distances from pivots[t] to every node.
 */
#ifndef SSM_H
#define SSM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSM_OK = 0,
    SSM_E_INVAL = 1,         /* bad argument or malformed graph */
    SSM_E_RANGE = 2,         /* size outside what the library supports */
    SSM_E_DISCONNECTED = 3,  /* a BFS did not reach every node */
    SSM_E_NOMEM = 4,         /* device allocation failed */
    SSM_E_DEVICE = 5         /* a HIP call failed */
} ssm_status;

typedef enum { SSM_FP64 = 0, SSM_FP32 = 1 } ssm_prec;

typedef enum { SSM_STRESS_SPARSE = 0, SSM_STRESS_FULL = 1, SSM_STRESS_NORMALIZED = 2 } ssm_stress_kind;

typedef struct {
    int32_t n;               /* nodes, >= 1 */
    int32_t nnz;             /* arcs = 2 m */
    const int32_t* row_ptr;  /* device [n+1] */
    const int32_t* col_idx;  /* device [nnz] */
} ssm_csr;

typedef struct ssm_terms ssm_terms; /* opaque, library-owned device state */

/* Checks on the device that g is a simple symmetric CSR: row_ptr monotone
 * from 0 to nnz, indices in range, no self-loop, no duplicate arc, every arc
 * matched by its reverse.  SSM_OK or SSM_E_INVAL.  Synchronizes. */
ssm_status ssm_validate_csr(const ssm_csr* g, hipStream_t stream);

/* Max/min shortest-path sampling (Section 4.1, "max/min sp"): pivots[0] =
 * first; pivots[t+1] is the node whose hop distance to the nearest of
 * pivots[0..t] is largest, the lowest node id on ties.  k in [1, n].
 * Writes pivots (device int32 [k]); if dist is not NULL also the k x n
 * distance table of those pivots.  SSM_E_DISCONNECTED if the graph is not
 * connected.  Synchronizes. */
ssm_status ssm_select_pivots(const ssm_csr* g, int32_t k, int32_t first, int32_t* pivots,
                             int32_t* dist, hipStream_t stream);

/* BFS from every pivot (the unweighted multi-source shortest paths of
 * Section 3, "Asymptotic running time") and the regions R(p) (Section 3):
 * dist (k x n), delta[i] = min_t dist[t][i] (distance to the nearest pivot),
 * region[i] = rank t of the pivot whose region holds i.  A node with one
 * nearest pivot joins it; ties favour the currently smallest region, read
 * level by level in delta: at level l the single-candidate nodes join first,
 * then each tied node joins the candidate with the smallest (size after
 * those joins, rank).  pivots must be distinct.  SSM_E_DISCONNECTED if a BFS
 * misses a node.  Synchronizes. */
ssm_status ssm_bfs_pivots(const ssm_csr* g, int32_t k, const int32_t* pivots, int32_t* dist,
                          int32_t* delta, int32_t* region, hipStream_t stream);

/* k-means sp (Section 4.1, "k-means sp"): refines the max/min pivots by
 * k-means over the nodes' hop-distance vectors y_i = (dist[0][i], ...,
 * dist[k-1][i]), the k x n table of those pivots (pivot-major).  Cluster t
 * starts as y_{pivots[t]}; each pass moves every node to the cluster whose
 * centroid (the mean of its members) is nearest, lowest rank on ties, then
 * recomputes the centroids (an empty cluster keeps its centroid); passes stop
 * when no node moves or after max_iters (the paper caps its k-means at 50).
 * new_pivots[t] is the node nearest to centroid t among the nodes not taken
 * by a lower rank, lowest id on ties.  The decisions run on exact integers:
 * clusters are integer sums S_t and sizes N_t, B_ti = y_i . S_t; a node
 * joins the t with the smallest a_t - (2 B_ti) / N_t, where
 * a_t = sum_j (S_tj / N_t)^2 is summed in ascending j in double without fused
 * multiply-add and the division is correctly rounded; the nearest node to a
 * centroid minimizes N_t ||y_i||^2 - 2 B_ti in 64-bit integers.
 * n, k: sizes (1 <= k <= n); pivots (device [k]): the max/min pivots;
 * dist (device [k][n]): their BFS rows; new_pivots (device [k]); assign
 * (device [n], may be NULL): the final cluster of every node;
 * iters_done_host (may be NULL): passes run.  The next step is
 * ssm_bfs_pivots with new_pivots.  SSM_E_RANGE if k n dmax^2 reaches 2^53.
 * Synchronizes. */
ssm_status ssm_kmeans_pivots(int32_t n, int32_t k, const int32_t* pivots, const int32_t* dist,
                             int32_t max_iters, int32_t* new_pivots, int32_t* assign,
                             int32_t* iters_done_host, hipStream_t stream);

/* Regions only, from a distance table already computed (same rule as
 * ssm_bfs_pivots).  Synchronizes. */
ssm_status ssm_regions(int32_t n, int32_t k, const int32_t* dist, int32_t* delta,
                       int32_t* region, hipStream_t stream);

/* Term set of Eq. 3 and Eq. 5 (Section 3, adapted weights): a pivot term
 * (i, t) exists iff dist[t][i] >= 2; its weight is w'_it = s / d^2 with
 * d = dist[t][i] and s = |{ j in R(pivots[t]) : delta_j <= floor(d / 2) }|,
 * i.e. the members of the region no farther from the pivot than half of d.
 * Builds the library-owned handle *out: a compressed copy of dist, the
 * cumulative region histograms H[t][l], the weight tables in FP64 and FP32
 * (FP64 by one correctly rounded division), the per-node denominators of
 * Eq. 5 (degree plus the pivot weights in ascending rank) and the scratch the
 * sweeps need.  Synchronizes.  Inputs are not retained. */
ssm_status ssm_build_terms(const ssm_csr* g, int32_t k, const int32_t* pivots,
                           const int32_t* dist, const int32_t* delta, const int32_t* region,
                           ssm_terms** out, hipStream_t stream);

void ssm_terms_free(ssm_terms* t);

/* Shape of a handle: k, delta_max (= max delta) and dmax (= max dist). */
ssm_status ssm_terms_dims(const ssm_terms* t, int32_t* k_host, int32_t* delta_max_host,
                          int32_t* dmax_host);

/* Copies tables out of a handle to host buffers (NULL skips one):
 * H [k][delta_max+1], wtab64 and wtab32 [k][dmax+1], den64 and den32 [n].
 * Synchronizes. */
ssm_status ssm_terms_export(const ssm_terms* t, int32_t* H_host, double* wtab64_host,
                            float* wtab32_host, double* den64_host, float* den32_host);

/* Algorithm 1, lines 3-4: PivotMDS start layout on the handle's pivots, then
 * a uniform rescale so that the summed layout length of the edges equals the
 * summed edge lengths (m).  PivotMDS: with S_ti = dist[t][i]^2, mu_t its mean
 * over nodes, nu_i its mean over pivots and gamma the mean of all entries,
 * C_it = -1/2 (S_ti - mu_t - nu_i + gamma); x = C V for V the eigenvectors of
 * the two largest eigenvalues of C^T C, each scaled so that its
 * largest-magnitude entry is positive.  Needs k >= 3.  x is written in the
 * precision p (the eigen step and the rescale run in FP64 either way).
 * Synchronizes. */
ssm_status ssm_pivotmds_init(const ssm_csr* g, ssm_terms* t, ssm_prec p, void* x,
                             hipStream_t stream);

/* Eigen data of the last ssm_pivotmds_init on this handle: V [k][2],
 * lambda [2], the iteration count of the eigen solver.  Synchronizes. */
ssm_status ssm_pivotmds_eig(const ssm_terms* t, double* V_host, double* lambda_host,
                            int32_t* iters_host);

/* The k x k Gram matrix C^T C of the last ssm_pivotmds_init on this handle
 * (row-major).  Synchronizes. */
ssm_status ssm_pivotmds_gram(const ssm_terms* t, double* M_host);

/* Algorithm 1, lines 5-8, with the update of Eq. 5 in Jacobi order (every
 * node reads the previous iterate): num_i = sum over neighbours j of
 * (x_j + (x_i - x_j)/r_ij) plus, over pivot terms, w'_it (x_p + d (x_i -
 * x_p)/r_ip); x_i <- num_i / den_i.  A vote whose distance r is 0 keeps only
 * x_q.  Runs `iters` sweeps in place on x (precision p); with tol > 0 stops
 * after the first sweep whose relative change ||x_new - x_old|| / ||x_old||
 * (Frobenius) is <= tol.  iters_done_host (may be NULL) receives the number
 * of sweeps run.  With tol == 0 the call is asynchronous unless
 * iters_done_host is given.  The FP64 form sums every node's terms in the
 * order stated (neighbours in CSR order, then pivots by ascending rank) with
 * correctly rounded square roots and divisions and no fused multiply-add. */
ssm_status ssm_majorize(const ssm_csr* g, ssm_terms* t, ssm_prec p, void* x, int32_t iters,
                        double tol, int32_t* iters_done_host, hipStream_t stream);

/* Mixed-precision sweeps: the first `warm` sweeps (1 <= warm) run in FP64
 * on the start layout x64 (in place); the layout is then rounded into x32 and
 * the remaining iters - warm sweeps run in FP32 on x32 (if iters <= warm, x32
 * just receives the rounded FP64 result).  The PivotMDS start places many
 * nodes within rounding distance of each other, where the update's
 * direction term (x_i - x_q) / r is ill-conditioned: rounding that start to
 * FP32 alone moves the final stress by ~1e-4, while rounding after one FP64
 * sweep moves it by ~1e-10.  Asynchronous. */
ssm_status ssm_majorize_mixed(const ssm_csr* g, ssm_terms* t, double* x64, float* x32, int32_t iters,
                              int32_t warm, hipStream_t stream);

/* Stress of layout x, accumulated in FP64: SSM_STRESS_SPARSE is s'(x) of
 * Eq. 3 (edges with w = 1, d = 1, plus every pivot term with w'_it);
 * SSM_STRESS_FULL is s(x) of Eq. 1 over all pairs with d the hop distance
 * and w = d^-2 (n <= 65536); SSM_STRESS_NORMALIZED is that full stress
 * divided by the number of pairs n (n - 1) / 2, the normalized stress of
 * Section 4.1 (n <= 65536, t may be NULL for both).  Writes out_host[0].
 * Synchronizes. */
ssm_status ssm_stress(const ssm_csr* g, ssm_terms* t, ssm_prec p, const void* x,
                      ssm_stress_kind kind, double* out_host, hipStream_t stream);

/* ---- Graphs with edge lengths (Algorithm 1's general input) ----------
 *
 * len (device, [nnz] doubles): a positive length per arc, equal on both arcs
 * of an edge.  d_ij is the shortest-path length, summed from the source
 * outwards in FP64 (the least solution of d(s) = 0, d(v) = min over
 * neighbours u of d(u) + len(u, v), exactly as Dijkstra's algorithm finds
 * it).  Edge terms carry w_ij = len^-2; a pivot term (i, p) exists for every
 * pivot p that is neither i nor a neighbour of i, with Section 3's weight
 * w'_ip = s / d_ip^2, s = |{ j in R(p) : d_jp <= d_ip / 2 }|, one weight per
 * (pivot, node).  Regions follow rule R1 with levels at the distinct values
 * of delta.  Unit lengths give the unweighted model's pivots, regions,
 * weights and FP64 sweeps exactly. */
typedef struct ssm_wterms ssm_wterms; /* opaque, library-owned device state */

/* max/min sp on lengths (Section 4.1): pivots[0] = first, each next pivot
 * the node farthest from the chosen ones (lowest id on ties); dist (may be
 * NULL) receives the k distance rows [k][n].  SSM_E_INVAL if a length is not
 * positive and finite (checked on the device before any search),
 * SSM_E_DISCONNECTED if a node is unreachable.  Synchronizes. */
ssm_status ssm_select_pivots_w(const ssm_csr* g, const double* len, int32_t k, int32_t first, int32_t* pivots,
                               double* dist, hipStream_t stream);
/* The k distance rows [k][n] of the given pivots (one label-correcting
 * search per pivot, in near-far bands of the largest length).  SSM_E_INVAL
 * if a length is not positive and finite.  Synchronizes. */
ssm_status ssm_sssp_pivots(const ssm_csr* g, const double* len, int32_t k, const int32_t* pivots, double* dist,
                           hipStream_t stream);
/* Regions, per-term weights and denominators (Section 3 with lengths) into a
 * new handle (copies pivots and dist).  Synchronizes. */
ssm_status ssm_build_terms_w(const ssm_csr* g, const double* len, int32_t k, const int32_t* pivots,
                             const double* dist, ssm_wterms** out, hipStream_t stream);
void ssm_wterms_free(ssm_wterms* t);
/* Copies delta [n], region [n], weights [k][n] and denominators [n] to host
 * buffers (each may be NULL). */
ssm_status ssm_wterms_export(const ssm_wterms* t, double* delta_host, int32_t* region_host, double* w_host,
                             double* den_host);
/* PivotMDS on the real distances, then the rescale to the summed edge
 * lengths (Algorithm 1's initialisation).  Synchronizes. */
ssm_status ssm_pivotmds_init_w(const ssm_csr* g, const double* len, const ssm_wterms* t, ssm_prec p, void* x,
                               hipStream_t stream);
/* iters Jacobi sweeps of Eq. 5 with lengths: FP64 in the oracle's order
 * (positive-distance neighbour votes in CSR order, the zero-distance ones,
 * then pivot terms by rank) or FP32 in displacement form.  Asynchronous. */
ssm_status ssm_majorize_w(const ssm_csr* g, const double* len, ssm_wterms* t, ssm_prec p, void* x, int32_t iters,
                          hipStream_t stream);
/* The first `warm` sweeps in FP64 on x64, rounded into x32, the rest in FP32
 * (as ssm_majorize_mixed).  Asynchronous. */
ssm_status ssm_majorize_mixed_w(const ssm_csr* g, const double* len, ssm_wterms* t, double* x64, float* x32,
                                int32_t iters, int32_t warm, hipStream_t stream);
/* s'(x) of Eq. 3 with lengths in FP64 into out_host[0].  Synchronizes. */
ssm_status ssm_stress_w(const ssm_csr* g, const double* len, const ssm_wterms* t, ssm_prec p, const void* x,
                        double* out_host, hipStream_t stream);

/* Procrustes statistic of layout x against the reference layout y (both
 * n x 2, interleaved, of precision px / py): the share of y's spread that x
 * misses after the best translation, rotation and dilation (no reflection),
 * the measure of Section 4.1 that compares a sparse layout with the
 * full-stress layout.  With X, Y centred and A = X^T Y:
 * 1 - (||A||_F^2 + 2 det A) / (tr(X^T X) tr(Y^T Y)), in [0, 1], 0 for a
 * perfect match.  Accumulated in FP64.  SSM_E_INVAL when a layout has all its
 * nodes at one point.  Writes out_host[0].  Synchronizes.
 * The paper's other measure, the normalized stress, is ssm_stress with
 * SSM_STRESS_NORMALIZED. */
ssm_status ssm_procrustes(int32_t n, ssm_prec px, const void* x, ssm_prec py, const void* y, double* out_host,
                          hipStream_t stream);

/* ssm_procrustes for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result bit for bit, with the partial sums
 * in a static device array of the library (6 x 1024 + 8 doubles, 49 KiB per
 * device, held until the process ends) instead of an allocated workspace.
 * It calls no allocating routine.  Every partial is written before it is
 * read, so nothing left by an earlier call is used.  All calls on one device
 * share that array: calls that overlap on one GPU (on different streams or
 * threads) race and must be serialized by the caller.  n in [2, 2^30]
 * (SSM_E_RANGE above); other errors as ssm_procrustes.  Synchronizes. */
ssm_status ssm_procrustes_noalloc(int32_t n, ssm_prec px, const void* x, ssm_prec py, const void* y,
                                  double* out_host, hipStream_t stream);

/* ---- Layout pool: many small graphs laid out together ----------------
 *
 * The same method (Algorithm 1: max/min sp pivots, their BFS, regions and
 * adapted weights of Section 3, PivotMDS, sweeps of Eq. 5) for many graphs
 * at once: every stage runs for a whole list of graphs per launch, and a
 * graph's CSR, packed distances, weight tables and coordinates stay resident
 * in one device arena of fixed capacity.  Graphs have 1 <= n <= 65536 nodes
 * and 3 <= k <= min(n, 256) pivots.  Calls on one pool are serialized
 * internally; a pool belongs to the device that was current at creation. */
typedef struct ssm_pool ssm_pool;

typedef enum {
    SSM_POOL_PIVOTS = 0,  /* int32 [k] */
    SSM_POOL_DIST = 1,    /* int32 [k][n] BFS distances of the pivots */
    SSM_POOL_DELTA = 2,   /* int32 [n] distance to the nearest pivot */
    SSM_POOL_REGION = 3,  /* int32 [n] region (pivot rank) */
    SSM_POOL_H = 4,       /* int32 [k][delta_max + 1] cumulative region histograms */
    SSM_POOL_WTAB64 = 5,  /* double [k][dmax + 1] adapted weights w'(t, d) */
    SSM_POOL_DEN64 = 6,   /* double [n] denominators of Eq. 5 */
    SSM_POOL_X32 = 7,     /* float [n][2] current layout */
    SSM_POOL_X64 = 8      /* double [n][2] FP64 layout after preparation (PivotMDS and the warm-up sweeps) */
} ssm_pool_table;

typedef enum { SSM_POOL_FREE = 0, SSM_POOL_ADDED = 1, SSM_POOL_READY = 2, SSM_POOL_FAILED = 3 } ssm_pool_state;

/* A pool with one device allocation of capacity_bytes (>= 1 MiB). */
ssm_status ssm_pool_create(int64_t capacity_bytes, ssm_pool** out);
void ssm_pool_destroy(ssm_pool* p);
/* Bytes of the arena in use and its capacity (host outputs, may be NULL). */
ssm_status ssm_pool_usage(ssm_pool* p, int64_t* used, int64_t* capacity);

/* Admits one graph: checks the host CSR's row pointers (monotone from 0 to
 * nnz) and ids (in [0, n)), reserves its resident and preparation buffers and
 * copies the CSR (row_ptr_host [n+1],
 * col_idx_host [nnz], host memory, read before return).  k pivots by max/min
 * from `first`; `sweeps` is the graph's total sweep count (Algorithm 1's
 * iteration bound).  SSM_E_NOMEM when the arena has no room: the caller may
 * retry after removing finished graphs (admission by memory budget).
 * Writes the slot id to *slot_out.  Synchronizes. */
ssm_status ssm_pool_add(ssm_pool* p, int32_t n, int32_t nnz, const int32_t* row_ptr_host,
                        const int32_t* col_idx_host, int32_t k, int32_t first, int32_t sweeps,
                        int32_t* slot_out, hipStream_t stream);

/* Preprocessing and start layout of the listed (added) slots: a check that
 * the graph is simple and undirected (no self-loop, repeated neighbour or
 * one-way arc; else the slot fails with SSM_E_INVAL), max/min
 * pivots, k BFS, regions (rule R1), H, w' and denominators, PivotMDS with the
 * rescale, then `warm` FP64 sweeps (oracle operation order), rounded into the
 * FP32 layout.  A slot whose graph is disconnected, has zero total PivotMDS
 * edge length or finds no room for its weight tables becomes
 * SSM_POOL_FAILED (see ssm_pool_info); the others become SSM_POOL_READY with
 * `warm` sweeps done.  Releases the preparation buffers.  Synchronizes. */
ssm_status ssm_pool_prepare(ssm_pool* p, int32_t count, const int32_t* slots_host, int32_t warm,
                            hipStream_t stream);

/* Up to `iters` FP32 Jacobi sweeps (Eq. 5, displacement form) on every
 * listed ready slot, never past its sweep count: one launch per sweep covers
 * all of them.  The quantum (its sweeps and stop tests) is one HIP graph,
 * captured once per rounded (chunks, graphs, sweeps, LDS) shape and
 * replayed; the kernels take the real counts from the staged header.  The
 * sweep runs a block per 256-node chunk or a persistent grid over the
 * chunks: the first call of a shape class times both (its first four sweeps)
 * and keeps the faster; the layouts do not depend on the choice.
 * Asynchronous; a later call that reads a slot (stress, layout, export,
 * remove) waits for it. */
ssm_status ssm_pool_sweep(ssm_pool* p, int32_t count, const int32_t* slots_host, int32_t iters,
                          hipStream_t stream);

/* s'(x) of Eq. 3 in FP64 for each listed ready slot's current layout into
 * out_host[count].  Synchronizes. */
ssm_status ssm_pool_stress(ssm_pool* p, int32_t count, const int32_t* slots_host, double* out_host,
                           hipStream_t stream);

/* Copies a ready slot's current FP32 layout (n x 2) to x_out (device). */
ssm_status ssm_pool_layout(ssm_pool* p, int32_t slot, float* x_out, hipStream_t stream);

/* Copies one table of a ready slot (ssm_pool_table) to host memory.
 * Synchronizes. */
ssm_status ssm_pool_export(ssm_pool* p, int32_t slot, int32_t what, void* host_out, hipStream_t stream);

/* info_host[8] = {state, failure status, n, k, sweeps done, sweep count,
 * dmax, delta_max}. */
ssm_status ssm_pool_info(ssm_pool* p, int32_t slot, int32_t* info_host);

/* Releases a slot's buffers (after any queued sweep that reads it). */
ssm_status ssm_pool_remove(ssm_pool* p, int32_t slot);

/* Stop test of Algorithm 1's loop for a slot's FP32 sweeps (ssm_pool_sweep):
 * after each sweep, the relative positional change (the change left after
 * the best rotation and translation of the previous iterate onto the new
 * one, over the previous iterate's spread about its centroid; FP64 moments)
 * is compared with tol; once it is at most tol the slot's layout stays at
 * that sweep's result (later sweeps of the slot carry it over unchanged).
 * tol = 0 (the default) runs the slot's sweep count.  The slot must be added
 * or ready. */
ssm_status ssm_pool_set_tol(ssm_pool* p, int32_t slot, double tol);

/* For each listed ready slot: sweeps_host[q] = the sweeps its layout took
 * (the FP64 warm-up sweeps included) if its stop test has fired, else -1.  A
 * stopped slot takes no further sweeps.  Waits for the pool's queued sweeps;
 * synchronizes. */
ssm_status ssm_pool_stopped(ssm_pool* p, int32_t count, const int32_t* slots, int32_t* sweeps_host,
                            hipStream_t stream);

/* Message for the last non-OK status returned on the calling thread. */
const char* ssm_last_error(void);

/* Returns the library's cached device scratch (buffers kept between calls
 * for reuse) to HIP, after synchronizing each device that holds some.
 * Handles (ssm_terms, ssm_wterms, ssm_pool) are not touched.  Meant for a
 * process that is about to exit, or that wants the memory back; later calls
 * allocate scratch again as needed.  Not to be called while another thread
 * runs a library call. */
void ssm_release_cache(void);

/* Forces a launch variant: another kernel form or launch shape of one step,
 * for tests and tuning experiments.  Every variant computes the same result
 * (integer outputs and FP64 sweeps bit for bit, FP32 sweeps within their
 * stated tolerance); only the speed changes.  value 0 restores the library's
 * own choice; name NULL clears every override.  The overrides are
 * process-wide; set them while no other thread runs a library call.
 * Names and values:
 *   select_mode 1|2|3|4 (one workgroup, cooperative grid over CSR rows,
 *   per-pivot launches, cooperative grid over padded rows),
 *   select_hyb 1 (in mode 4: each pruned BFS by one block of the grid,
 *   the argmax by all of it),
 *   select_blocks N, select_threads 256|512, select_ell 2 (plain CSR),
 *   select_m8 2 (no LDS byte copy), select_rowq 2, select_pre 1|3,
 *   select_wave -1|2 (block levels only, two passes per wave level),
 *   bfs_ell 2|3|4 (CSR rows; padded rows with the distance row as visited
 *   set, with or without a read before the swap), bfs_rowq 2,
 *   bfs_loads 2|3 (CSR rows: plain visited checks as well as plain CSR
 *   loads, or agent-scope loads throughout), bfs_grp -1 (CSR rows on one
 *   workgroup each instead of two),
 *   bfs_lanes 2..64, msbfs -1|1 (never / always the bit-parallel BFS
 *   first; by default it goes first on graphs of at least 2^19 arcs whose
 *   mean neighbour degree is at least 3x their mean degree), msbfs_budget N,
 *   region_mode 1|2, km_chunk 32|40|48|56|64,
 *   sweep_mode 1|2 (LDS histograms, global table), sweep_split 1|2|4,
 *   sweep_blocks_per_cu N, sweep_waves 4|16 (waves per block),
 *   sweep_tune -1 (no timing of launch shapes: the rule shape; the FP32
 *   sweep otherwise times its shapes on the first loop of at least 24
 *   sweeps per graph shape and keeps the fastest),
 *   sweep_perm -1|2 (caller's node order, always reorder),
 *   sweep_f64_terms -1 (FP64 sweeps of small graphs one thread per node
 *   instead of a lane group per node; same result),
 *   sssp_nearfar -1 (plain rounds), sssp_band N,
 *   ell_width 8|16|32 (slots per padded adjacency row in BFS and selection),
 *   pool_graph -1 (ssm_pool_sweep launches each kernel instead of replaying
 *   a captured HIP graph of the quantum), pool_persist 1|-1 (the pooled
 *   sweep on a persistent grid, or a block per chunk, instead of the timed
 *   choice).
 * SSM_E_INVAL for an unknown name. */
ssm_status ssm_set_variant(const char* name, int32_t value);

#ifdef __cplusplus
}
#endif
#endif /* SSM_H */
