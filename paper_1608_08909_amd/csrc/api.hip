// C ABI entry points of libssm: argument checks, error reporting, dispatch.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "ssm_internal.h"

namespace ssm {

static thread_local std::string g_last_error;

ssm_status fail(ssm_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

ssm_status hip_fail(hipError_t e, const char* what) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s", what, hipGetErrorString(e));
    if (e == hipErrorOutOfMemory) return fail(SSM_E_NOMEM, buf);
    return fail(SSM_E_DEVICE, buf);
}

ssm_status dalloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        char buf[160];
        snprintf(buf, sizeof buf, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
        return fail(e == hipErrorOutOfMemory ? SSM_E_NOMEM : SSM_E_DEVICE, buf);
    }
    return SSM_OK;
}

// Scratch cache: buffers released by sfree stay allocated and serve later
// salloc calls of at most four times smaller size on the same device, up to
// kScratchCacheBytes in total (the largest are released first beyond it).
// Every caller releases scratch only after synchronizing the stream that
// used it, so a cached buffer is idle when it is handed out again.
namespace {
struct CachedBlock {
    int dev;
    void* p;
    size_t bytes;
};
std::mutex g_scratch_mu;
std::vector<CachedBlock> g_scratch_free;
std::unordered_map<void*, CachedBlock> g_scratch_live;
size_t g_scratch_free_bytes = 0;
constexpr size_t kScratchCacheBytes = 8ull << 30;
constexpr size_t kScratchGrain = 2u << 20;
}  // namespace

ssm_status salloc(void** p, size_t bytes) {
    *p = nullptr;
    int dev = 0;
    (void)hipGetDevice(&dev);
    bytes = std::max<size_t>(bytes, 16);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    int best = -1;
    for (int q = 0; q < (int)g_scratch_free.size(); ++q) {
        const CachedBlock& b = g_scratch_free[q];
        if (b.dev == dev && b.bytes >= bytes && b.bytes / 4 <= bytes &&
            (best < 0 || b.bytes < g_scratch_free[best].bytes))
            best = q;
    }
    if (best >= 0) {
        CachedBlock b = g_scratch_free[best];
        g_scratch_free.erase(g_scratch_free.begin() + best);
        g_scratch_free_bytes -= b.bytes;
        g_scratch_live[b.p] = b;
        *p = b.p;
        return SSM_OK;
    }
    const size_t rounded = (bytes + kScratchGrain - 1) / kScratchGrain * kScratchGrain;
    ssm_status st = dalloc(p, rounded);
    if (st != SSM_OK) return st;
    g_scratch_live[*p] = CachedBlock{dev, *p, rounded};
    return SSM_OK;
}

void sfree(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_live.find(p);
    if (it == g_scratch_live.end()) {
        (void)hipFree(p);
        return;
    }
    g_scratch_free.push_back(it->second);
    g_scratch_free_bytes += it->second.bytes;
    g_scratch_live.erase(it);
    while (g_scratch_free_bytes > kScratchCacheBytes) {
        auto big = std::max_element(g_scratch_free.begin(), g_scratch_free.end(),
                                    [](const CachedBlock& a, const CachedBlock& b) { return a.bytes < b.bytes; });
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(big->dev);
        (void)hipFree(big->p);
        (void)hipSetDevice(cur);
        g_scratch_free_bytes -= big->bytes;
        g_scratch_free.erase(big);
    }
}

// Returns every cached (idle) scratch block to HIP.  Live blocks stay with
// their owners.  Each device that holds cached blocks is synchronized first.
void release_cached_scratch() {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_free.empty()) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (const CachedBlock& b : g_scratch_free) {
        (void)hipSetDevice(b.dev);
        (void)hipDeviceSynchronize();
        (void)hipFree(b.p);
    }
    g_scratch_free.clear();
    g_scratch_free_bytes = 0;
    (void)hipSetDevice(cur);
}

// Launch-variant overrides (set through ssm_set_variant; 0 or absent = the
// library's own choice).  Process-wide, guarded by a mutex.
namespace {
std::mutex g_variant_mu;
std::unordered_map<std::string, int> g_variants;
const char* const kVariantNames[] = {
    "bfs_lanes",   "bfs_rowq",      "bfs_ell",       "msbfs",         "msbfs_budget", "select_threads",
    "select_wave", "select_rowq",   "select_pre",    "select_blocks", "select_mode",  "select_ell", "select_hyb",
    "select_m8",   "region_mode",   "km_chunk",      "sweep_perm",    "sweep_mode",   "sweep_split",
    "sweep_blocks_per_cu", "sweep_waves", "sweep_tune", "sssp_nearfar", "sssp_band", "ell_width", "pool_graph", "pool_persist", "sweep_f64_terms", "bfs_loads", "bfs_grp"};
}  // namespace

int variant(const char* name, int unset) {
    std::lock_guard<std::mutex> lock(g_variant_mu);
    auto it = g_variants.find(name);
    return it == g_variants.end() ? unset : it->second;
}

ssm_status check_csr(const ssm_csr* g) {
    if (!g) return fail(SSM_E_INVAL, "graph is NULL");
    if (g->n < 1) return fail(SSM_E_INVAL, "graph has no nodes");
    if (g->nnz < 0) return fail(SSM_E_INVAL, "negative arc count");
    if (!g->row_ptr || (g->nnz > 0 && !g->col_idx))
        return fail(SSM_E_INVAL, "graph pointers are NULL");
    if (g->n > (1 << 30)) return fail(SSM_E_RANGE, "n above 2^30");
    return SSM_OK;
}

int num_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    return cus;
}

}  // namespace ssm

using namespace ssm;

extern "C" {

const char* ssm_last_error(void) { return g_last_error.c_str(); }

void ssm_release_cache(void) { release_cached_scratch(); }

ssm_status ssm_set_variant(const char* name, int32_t value) {
    if (!name) {  // clear every override
        std::lock_guard<std::mutex> lock(g_variant_mu);
        g_variants.clear();
        return SSM_OK;
    }
    bool known = false;
    for (const char* v : kVariantNames) known = known || strcmp(v, name) == 0;
    if (!known) return fail(SSM_E_INVAL, std::string("unknown variant name: ") + name);
    std::lock_guard<std::mutex> lock(g_variant_mu);
    if (value == 0)
        g_variants.erase(name);
    else
        g_variants[name] = value;
    return SSM_OK;
}

ssm_status ssm_select_pivots(const ssm_csr* g, int32_t k, int32_t first, int32_t* pivots,
                             int32_t* dist, hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (k < 1 || k > g->n) return fail(SSM_E_INVAL, "k must lie in [1, n]");
    if (first < 0 || first >= g->n) return fail(SSM_E_INVAL, "first must lie in [0, n)");
    if (!pivots) return fail(SSM_E_INVAL, "pivots is NULL");
    if ((long long)k * g->n >= (1LL << 40)) return fail(SSM_E_RANGE, "k * n too large");
    st = select_pivots(g, k, first, pivots, stream);
    if (st != SSM_OK || !dist) return st;
    int32_t dmax = 0;
    return mssp(g, k, pivots, dist, &dmax, stream);
}

ssm_status ssm_bfs_pivots(const ssm_csr* g, int32_t k, const int32_t* pivots, int32_t* dist,
                          int32_t* delta, int32_t* region, hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (k < 1 || k > g->n) return fail(SSM_E_INVAL, "k must lie in [1, n]");
    if (!pivots || !dist || !delta || !region) return fail(SSM_E_INVAL, "NULL output or pivots");
    if ((long long)k * g->n >= (1LL << 40)) return fail(SSM_E_RANGE, "k * n too large");
    int32_t dmax = 0;
    st = mssp(g, k, pivots, dist, &dmax, stream);
    if (st != SSM_OK) return st;
    return regions(g->n, k, dist, delta, region, stream);
}

ssm_status ssm_kmeans_pivots(int32_t n, int32_t k, const int32_t* pivots, const int32_t* dist,
                             int32_t max_iters, int32_t* new_pivots, int32_t* assign, int32_t* iters_done_host,
                             hipStream_t stream) {
    if (n < 1 || k < 1 || k > n) return fail(SSM_E_INVAL, "need 1 <= k <= n");
    if (max_iters < 1) return fail(SSM_E_INVAL, "max_iters must be at least 1");
    if (!pivots || !dist || !new_pivots) return fail(SSM_E_INVAL, "NULL pointer");
    if ((long long)k * n >= (1LL << 40)) return fail(SSM_E_RANGE, "k * n too large");
    return kmeans_pivots(n, k, pivots, dist, max_iters, new_pivots, assign, iters_done_host, stream);
}

ssm_status ssm_regions(int32_t n, int32_t k, const int32_t* dist, int32_t* delta, int32_t* region,
                       hipStream_t stream) {
    if (n < 1 || k < 1 || k > n) return fail(SSM_E_INVAL, "need 1 <= k <= n");
    if (!dist || !delta || !region) return fail(SSM_E_INVAL, "NULL pointer");
    return regions(n, k, dist, delta, region, stream);
}

ssm_status ssm_build_terms(const ssm_csr* g, int32_t k, const int32_t* pivots,
                           const int32_t* dist, const int32_t* delta, const int32_t* region,
                           ssm_terms** out, hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!out) return fail(SSM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (k < 1 || k > g->n) return fail(SSM_E_INVAL, "k must lie in [1, n]");
    if (!pivots || !dist || !delta || !region) return fail(SSM_E_INVAL, "NULL input");
    return build_terms(g, k, pivots, dist, delta, region, out, stream);
}

void ssm_terms_free(ssm_terms* t) {
    if (!t) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(t->device);
    // the arena and the heavy-row lists come from the scratch cache: returned
    // only once the device is idle
    (void)hipDeviceSynchronize();
    sfree(t->arena);
    void* ptrs[] = {t->heavy, t->seg_start, t->seg_owner, t->seg_range, t->seg_sum};
    for (void* p : ptrs) sfree(p);
    (void)hipSetDevice(cur);
    delete t;
}

ssm_status ssm_terms_dims(const ssm_terms* t, int32_t* k_host, int32_t* delta_max_host,
                          int32_t* dmax_host) {
    if (!t) return fail(SSM_E_INVAL, "terms is NULL");
    if (k_host) *k_host = t->k;
    if (delta_max_host) *delta_max_host = t->delta_max;
    if (dmax_host) *dmax_host = t->dmax;
    return SSM_OK;
}

ssm_status ssm_terms_export(const ssm_terms* t, int32_t* H_host, double* wtab64_host,
                            float* wtab32_host, double* den64_host, float* den32_host) {
    if (!t) return fail(SSM_E_INVAL, "terms is NULL");
    SSM_HIP(hipDeviceSynchronize());
    size_t kw = (size_t)t->k * t->W;
    if (H_host)
        SSM_HIP(hipMemcpy(H_host, t->H, sizeof(int32_t) * (size_t)t->k * (t->delta_max + 1),
                          hipMemcpyDeviceToHost));
    if (wtab64_host)
        SSM_HIP(hipMemcpy(wtab64_host, t->wtab64, sizeof(double) * kw, hipMemcpyDeviceToHost));
    if (wtab32_host)
        SSM_HIP(hipMemcpy(wtab32_host, t->wtab32, sizeof(float) * kw, hipMemcpyDeviceToHost));
    if (den64_host)
        SSM_HIP(hipMemcpy(den64_host, t->den64, sizeof(double) * t->n, hipMemcpyDeviceToHost));
    if (den32_host)
        SSM_HIP(hipMemcpy(den32_host, t->den32, sizeof(float) * t->n, hipMemcpyDeviceToHost));
    return SSM_OK;
}

ssm_status ssm_pivotmds_init(const ssm_csr* g, ssm_terms* t, ssm_prec p, void* x,
                             hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!t || !x) return fail(SSM_E_INVAL, "NULL terms or layout");
    if (t->n != g->n) return fail(SSM_E_INVAL, "terms were built for another graph");
    if (p != SSM_FP64 && p != SSM_FP32) return fail(SSM_E_INVAL, "unknown precision");
    if (t->k < 3) return fail(SSM_E_INVAL, "PivotMDS needs k >= 3");
    return pivotmds(g, t, p, x, stream);
}

ssm_status ssm_pivotmds_eig(const ssm_terms* t, double* V_host, double* lambda_host,
                            int32_t* iters_host) {
    if (!t) return fail(SSM_E_INVAL, "terms is NULL");
    SSM_HIP(hipDeviceSynchronize());
    if (V_host)
        SSM_HIP(hipMemcpy(V_host, t->eig, sizeof(double) * 2 * t->k, hipMemcpyDeviceToHost));
    if (lambda_host)
        SSM_HIP(hipMemcpy(lambda_host, t->eig + 2 * t->k, sizeof(double) * 2,
                          hipMemcpyDeviceToHost));
    if (iters_host)
        SSM_HIP(hipMemcpy(iters_host, t->eig_iters, sizeof(int32_t), hipMemcpyDeviceToHost));
    return SSM_OK;
}

ssm_status ssm_pivotmds_gram(const ssm_terms* t, double* M_host) {
    if (!t || !M_host) return fail(SSM_E_INVAL, "NULL argument");
    SSM_HIP(hipDeviceSynchronize());
    SSM_HIP(hipMemcpy(M_host, t->gram, sizeof(double) * (size_t)t->k * t->k, hipMemcpyDeviceToHost));
    return SSM_OK;
}

ssm_status ssm_majorize(const ssm_csr* g, ssm_terms* t, ssm_prec p, void* x, int32_t iters,
                        double tol, int32_t* iters_done_host, hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!t || !x) return fail(SSM_E_INVAL, "NULL terms or layout");
    if (t->n != g->n || t->nnz != g->nnz) return fail(SSM_E_INVAL, "terms were built for another graph");
    if (p != SSM_FP64 && p != SSM_FP32) return fail(SSM_E_INVAL, "unknown precision");
    if (iters < 0) return fail(SSM_E_INVAL, "negative iteration count");
    if (!(tol >= 0.0)) return fail(SSM_E_INVAL, "tol must be >= 0");
    return majorize(g, t, p, x, iters, tol, iters_done_host, stream);
}

ssm_status ssm_majorize_mixed(const ssm_csr* g, ssm_terms* t, double* x64, float* x32, int32_t iters,
                              int32_t warm, hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!t || !x64 || !x32) return fail(SSM_E_INVAL, "NULL terms or layout");
    if (t->n != g->n || t->nnz != g->nnz) return fail(SSM_E_INVAL, "terms were built for another graph");
    if (iters < 0) return fail(SSM_E_INVAL, "negative iteration count");
    if (warm < 1) return fail(SSM_E_INVAL, "warm must be >= 1");
    return majorize_mixed(g, t, x64, x32, iters, warm, stream);
}

ssm_status ssm_stress(const ssm_csr* g, ssm_terms* t, ssm_prec p, const void* x,
                      ssm_stress_kind kind, double* out_host, hipStream_t stream) {
    ssm_status st = check_csr(g);
    if (st != SSM_OK) return st;
    if (!x || !out_host) return fail(SSM_E_INVAL, "NULL layout or output");
    if (p != SSM_FP64 && p != SSM_FP32) return fail(SSM_E_INVAL, "unknown precision");
    if (kind == SSM_STRESS_SPARSE) {
        if (!t) return fail(SSM_E_INVAL, "sparse stress needs terms");
        if (t->n != g->n) return fail(SSM_E_INVAL, "terms were built for another graph");
        return stress_sparse(g, t, p, x, out_host, stream);
    }
    if (kind == SSM_STRESS_FULL || kind == SSM_STRESS_NORMALIZED) {
        if (g->n > 65536) return fail(SSM_E_RANGE, "full stress supports n <= 65536");
        st = stress_full(g, p, x, out_host, stream);
        // normalized stress (Section 4.1): per node pair
        if (st == SSM_OK && kind == SSM_STRESS_NORMALIZED) out_host[0] /= (double)g->n * (g->n - 1) / 2.0;
        return st;
    }
    return fail(SSM_E_INVAL, "unknown stress kind");
}

ssm_status ssm_procrustes(int32_t n, ssm_prec px, const void* x, ssm_prec py, const void* y, double* out_host,
                          hipStream_t stream) {
    if (n < 2) return fail(SSM_E_INVAL, "need n >= 2");
    if (!x || !y || !out_host) return fail(SSM_E_INVAL, "NULL layout or output");
    if ((px != SSM_FP64 && px != SSM_FP32) || (py != SSM_FP64 && py != SSM_FP32))
        return fail(SSM_E_INVAL, "unknown precision");
    return procrustes(n, px, x, py, y, out_host, stream);
}

ssm_status ssm_procrustes_noalloc(int32_t n, ssm_prec px, const void* x, ssm_prec py, const void* y,
                                  double* out_host, hipStream_t stream) {
    if (n < 2) return fail(SSM_E_INVAL, "need n >= 2");
    if (n > (1 << 30)) return fail(SSM_E_RANGE, "n above 2^30");
    if (!x || !y || !out_host) return fail(SSM_E_INVAL, "NULL layout or output");
    if ((px != SSM_FP64 && px != SSM_FP32) || (py != SSM_FP64 && py != SSM_FP32))
        return fail(SSM_E_INVAL, "unknown precision");
    return procrustes_noalloc(n, px, x, py, y, out_host, stream);
}

}  // extern "C"
