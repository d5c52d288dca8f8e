// Layout quality measures of the paper's evaluation (Section 4.1): the
// Procrustes statistic of a layout against a reference layout, matching by
// translation, rotation and dilation (no reflection).
//
// With X and Y the centred n x 2 layouts and A = X^T Y, the best rotation R
// maximizes tr(R A); for 2 x 2 matrices restricted to proper rotations that
// maximum is sigma_1 + sign(det A) sigma_2 = sqrt(||A||_F^2 + 2 det A), so
//     statistic = 1 - (||A||_F^2 + 2 det A) / (tr(X^T X) tr(Y^T Y)),
// in [0, 1], 0 for a perfect match.  Two passes in FP64: the means, then the
// centred second moments, each as per-block partials summed in a fixed order.
#include <mutex>
#include <unordered_map>

#include "ssm_internal.h"
#include "wave.h"

namespace ssm {

constexpr int kQMaxBlocks = 1024;                          // blocks of one pass (grid-stride beyond)
constexpr size_t kQScratch = 6 * (size_t)kQMaxBlocks + 8;  // doubles: partials, means, statistic, flag

// Scratch of the allocation-free entry point: one copy per device, held
// until the process ends.  Host code never passes the symbol itself to a
// kernel; it uses the device address looked up once per device below.
static __device__ __align__(256) double scratch[kQScratch];

template <typename T2>
__device__ __forceinline__ double2 q_load(const void* p, int i) {
    const T2 v = ((const T2*)p)[i];
    return make_double2((double)v.x, (double)v.y);
}

__device__ __forceinline__ double2 q_at(int prec, const void* p, int i) {
    return prec == SSM_FP64 ? q_load<double2>(p, i) : q_load<float2>(p, i);
}

constexpr int kQBlock = 256;

// pass 0: partials of (sum x, sum y) into part[b][4]; pass 1: of the
// centred moments (xx, yy, A00, A01, A10, A11) into part[b][6], with the
// means from mean[4].
template <int PASS>
__global__ __launch_bounds__(kQBlock) void k_procrustes(int n, int px, const void* x, int py, const void* y,
                                                        const double* __restrict__ mean,
                                                        double* __restrict__ part) {
    constexpr int V = PASS == 0 ? 4 : 6;
    double acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0;
    double mx0 = 0.0, mx1 = 0.0, my0 = 0.0, my1 = 0.0;
    if (PASS == 1) {
        mx0 = mean[0];
        mx1 = mean[1];
        my0 = mean[2];
        my1 = mean[3];
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double2 a = q_at(px, x, i), b = q_at(py, y, i);
        if (PASS == 0) {
            acc[0] += a.x;
            acc[1] += a.y;
            acc[2] += b.x;
            acc[3] += b.y;
        } else {
            const double a0 = a.x - mx0, a1 = a.y - mx1, b0 = b.x - my0, b1 = b.y - my1;
            acc[0] += a0 * a0 + a1 * a1;
            acc[1] += b0 * b0 + b1 * b1;
            acc[2] += a0 * b0;
            acc[3] += a0 * b1;
            acc[4] += a1 * b0;
            acc[5] += a1 * b1;
        }
    }
    __shared__ double red[kQBlock / kWave];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const double s = block_sum(acc[v], red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * V + v] = s;
    }
}

// One thread: the partials in block order; PASS 0 writes the means, PASS 1
// the statistic (out[0]) and a flag (out[1] = 1 when a layout has no spread).
template <int PASS>
__global__ void k_procrustes_final(int n, int nb, const double* __restrict__ part, double* __restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    constexpr int V = PASS == 0 ? 4 : 6;
    double s[V];
    for (int v = 0; v < V; ++v) s[v] = 0.0;
    for (int b = 0; b < nb; ++b)
        for (int v = 0; v < V; ++v) s[v] += part[(size_t)b * V + v];
    if (PASS == 0) {
        for (int v = 0; v < 4; ++v) out[v] = s[v] / (double)n;
    } else {
        const double fro = s[2] * s[2] + s[3] * s[3] + s[4] * s[4] + s[5] * s[5];
        const double det = s[2] * s[5] - s[3] * s[4];
        const double den = s[0] * s[1];
        out[1] = den > 0.0 ? 0.0 : 1.0;
        out[0] = den > 0.0 ? 1.0 - (fro + 2.0 * det) / den : 0.0;
    }
}

// The two passes on workspace ws (at least 6 nb + 8 doubles, nb the block
// count below); every partial is written before it is read.
static ssm_status procrustes_ws(int32_t n, int32_t px, const void* x, int32_t py, const void* y, double* out_host,
                                hipStream_t s, double* ws) {
    const int nb = std::max(1, std::min(div_up(n, kQBlock), kQMaxBlocks));
    double* part = ws;
    double* res = ws + 6 * (size_t)nb;  // means [4], then statistic and flag
    hipLaunchKernelGGL(k_procrustes<0>, dim3(nb), dim3(kQBlock), 0, s, n, px, x, py, y, res, part);
    hipLaunchKernelGGL(k_procrustes_final<0>, dim3(1), dim3(64), 0, s, n, nb, part, res);
    hipLaunchKernelGGL(k_procrustes<1>, dim3(nb), dim3(kQBlock), 0, s, n, px, x, py, y, res, part);
    hipLaunchKernelGGL(k_procrustes_final<1>, dim3(1), dim3(64), 0, s, n, nb, part, res + 4);
    hipError_t e = hipGetLastError();
    double h[2] = {0.0, 0.0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, res + 4, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "Procrustes statistic");
    if (h[1] != 0.0) return fail(SSM_E_INVAL, "a layout has all nodes at one point");
    *out_host = h[0];
    return SSM_OK;
}

ssm_status procrustes(int32_t n, int32_t px, const void* x, int32_t py, const void* y, double* out_host,
                      hipStream_t s) {
    double* ws = nullptr;
    ssm_status st = salloc((void**)&ws, sizeof(double) * kQScratch);
    if (st != SSM_OK) return st;
    st = procrustes_ws(n, px, x, py, y, out_host, s, ws);  // synchronizes s before returning
    sfree(ws);
    return st;
}

// Device address of `scratch` on the current device, looked up on the
// first call on that device.
static ssm_status scratch_address(double** out) {
    static std::mutex mu;
    static std::unordered_map<int, double*> addr;
    int dev = 0;
    SSM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) {
        *out = it->second;
        return SSM_OK;
    }
    double* p = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    addr[dev] = p;
    *out = p;
    return SSM_OK;
}

ssm_status procrustes_noalloc(int32_t n, int32_t px, const void* x, int32_t py, const void* y, double* out_host,
                              hipStream_t s) {
    double* ws = nullptr;
    ssm_status st = scratch_address(&ws);
    if (st != SSM_OK) return st;
    return procrustes_ws(n, px, x, py, y, out_host, s, ws);
}

}  // namespace ssm
