// Localized majorization sweeps (paper Eq. 5, Algorithm 1 lines 5-8) in
// Jacobi order, and the stress of Eq. 3 and Eq. 1.
#include <float.h>
#include <math.h>
#include <stdlib.h>

#include <vector>

#include "ssm_internal.h"
#include "wave.h"

namespace ssm {

// ------------------------------------------------------------- reductions

// out[0] = sum of partials[0..count) in a fixed order (one block).
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partials, int count,
                                                      double* __restrict__ out) {
    double s = 0.0;
    for (int q = threadIdx.x; q < count; q += blockDim.x) s += partials[q];
    __shared__ double red[256 / kWave];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[0] = s;
}

void launch_sum_partials(const double* partials, int count, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, count, out);
}

template <typename DT, int VEC>
union Packed {
    uint4 v;
    DT e[VEC];
};

// --------------------------------------------------------- FP64 sweep

// One thread per node.  Terms are summed exactly in the order stated by the
// update: neighbours at a positive distance in CSR order (w = 1, d = 1), then
// the neighbours at distance zero (each votes x_q = x_i), then pivot terms in
// ascending rank; vote(q, d) = x_q + (d (x_i - x_q)) / r, or x_q when r = 0;
// correctly rounded sqrt and division, no contraction into fused
// multiply-adds.  x_new_i = num / den_i.
template <typename DT, int VEC>
__global__ __launch_bounds__(256) void k_sweep_f64(int n, int kpad, int W, const int* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const double2* __restrict__ xo,
                                                   double2* __restrict__ xn, const uint4* __restrict__ dpk,
                                                   const int* __restrict__ piv,
                                                   const double* __restrict__ wt,
                                                   const double* __restrict__ den) {
#pragma clang fp contract(off)
    extern __shared__ double2 sP[];
    for (int t = threadIdx.x; t < kpad; t += blockDim.x) sP[t] = xo[piv[t]];
    __syncthreads();
    const int nwords = kpad / VEC;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double2 xv = xo[i];
        const double xi = xv.x, yi = xv.y;
        double nx = 0.0, ny = 0.0;
        int zero = 0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const double2 xj = xo[ci[e]];
            double dx = xi - xj.x, dy = yi - xj.y;
            double r = sqrt(dx * dx + dy * dy);
            if (r > 0.0) {
                nx += xj.x + dx / r;
                ny += xj.y + dy / r;
            } else {
                ++zero;
            }
        }
        for (int z = 0; z < zero; ++z) {
            nx += xi;
            ny += yi;
        }
        for (int b = 0; b < nwords; ++b) {
            Packed<DT, VEC> u;
            u.v = dpk[(size_t)b * n + i];
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const int d = (int)u.e[j];
                if (d < 2) continue;
                const int t = b * VEC + j;
                const double w = wt[(size_t)t * W + d];
                const double2 p = sP[t];
                double dx = xi - p.x, dy = yi - p.y;
                double r = sqrt(dx * dx + dy * dy);
                double vx = p.x, vy = p.y;
                if (r > 0.0) {
                    vx = p.x + (double)d * dx / r;
                    vy = p.y + (double)d * dy / r;
                }
                nx += w * vx;
                ny += w * vy;
            }
        }
        const double dn = den[i];
        xn[i] = make_double2(nx / dn, ny / dn);
    }
}

// --------------------------------------------------------- FP32 sweep

// How the FP32 sweep finds (w', w' d) for a pivot term.
enum WeightMode { kTableLds = 0, kHistLds = 1, kTableGlobal = 2 };

// Eq. 5 in displacement form: x_i' = x_i + (sum_q f_q (x_q - x_i)) / den_i
// with f_q = w_q - (w_q d_q) / r_iq, which equals num_i / den_i because every
// vote minus x_i is (x_q - x_i)(1 - d_q / r_iq).  Accumulating displacements
// keeps FP32 rounding relative to the (small) move rather than to the
// coordinates, and a vote at distance zero contributes exactly 0, so two
// coincident nodes with one closed neighbourhood get identical updates.
//
// Block = WAVES wavefronts over 64 consecutive nodes (lane = node): wave w
// sums the packed distance words b = w, w + WAVES, ... (one coalesced 16-byte
// load per lane covers VEC pivots; every lane of the wave reads the same
// pivot, so its coordinates and table row come from LDS as broadcasts);
// the last wave (fewest words) also sums the neighbour terms in CSR order.  The WAVES partials are
// added in a fixed order.  Weights: kTableLds stages (w', w'd) for every
// (pivot, distance); kHistLds stages the region histograms H and (1/d^2, 1/d)
// and forms w' = H[t][min(d/2, delta_max)] / d^2; kTableGlobal reads the table
// from memory.  1/r is the hardware reciprocal square root of r^2 + 1e-30.
// Neighbour displacement sums of the high-degree nodes, one wavefront each:
// lane l sums the neighbours e = l, l + 64, ... of its row in order, then the
// 64 partials are combined by a fixed butterfly.  Same terms as the FP32
// sweep's neighbour loop: (1 - 1/r) (x_j - x_i).
__global__ __launch_bounds__(256) void k_heavy_edges(int nheavy, const int* __restrict__ heavy,
                                                     const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const float2* __restrict__ xo, float2* __restrict__ out) {
    const int lane = lane_id();
    const float tiny = 1e-30f;
    for (int h = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; h < nheavy;
         h += gridDim.x * blockDim.x / kWave) {
        const int i = heavy[h];
        const float2 xi = xo[i];
        float ax = 0.f, ay = 0.f;
        for (int e = rp[i] + lane; e < rp[i + 1]; e += kWave) {
            const float2 xj = xo[ci[e]];
            float dx = xj.x - xi.x, dy = xj.y - xi.y;
            float f = 1.f - __builtin_amdgcn_rsqf(dx * dx + (dy * dy + tiny));
            ax += f * dx;
            ay += f * dy;
        }
        ax = wave_sum(ax);
        ay = wave_sum(ay);
        if (lane == 0) out[h] = make_float2(ax, ay);
    }
}

// Position of node i in the ascending heavy list (binary search).
__device__ __forceinline__ int heavy_index(const int* __restrict__ heavy, int nheavy, int i) {
    int lo = 0, hi = nheavy - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (heavy[mid] < i)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <typename DT, int VEC, int WAVES, int MODE>
__global__ __launch_bounds__(64 * WAVES) void k_sweep_f32(
    int n, int kpad, int W, int L, const int* __restrict__ rp, const int* __restrict__ ci,
    const float2* __restrict__ xo, float2* __restrict__ xn, const uint4* __restrict__ dpk,
    const int* __restrict__ piv, const float2* __restrict__ wt2, const float* __restrict__ Hf,
    const float2* __restrict__ invd, const float* __restrict__ den, const int* __restrict__ heavy, int nheavy,
    const float2* __restrict__ heavy_sum) {
    extern __shared__ float4 smem4[];
    float2* sP = (float2*)smem4;                 // [kpad]
    float2* sPart = sP + kpad;                   // [WAVES][64]
    float2* sTab = sPart + WAVES * 64;           // kTableLds: [kpad][W]; kHistLds: invd [W]
    float* sH = (float*)(sTab + (MODE == kHistLds ? W : 0));  // kHistLds: [kpad][L]
    for (int t = threadIdx.x; t < kpad; t += blockDim.x) sP[t] = xo[piv[t]];
    if (MODE == kTableLds)
        for (int q = threadIdx.x; q < kpad * W; q += blockDim.x) sTab[q] = wt2[q];
    if (MODE == kHistLds) {
        for (int q = threadIdx.x; q < W; q += blockDim.x) sTab[q] = invd[q];
        for (int q = threadIdx.x; q < kpad * L; q += blockDim.x) sH[q] = Hf[q];
    }
    __syncthreads();
    const int lane = threadIdx.x % 64;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);  // wave-uniform
    const int nwords = kpad / VEC;
    // r^2 gets 1e-30 added: a vote at distance zero then has a finite factor
    // times a zero displacement, i.e. contributes exactly 0
    const float tiny = 1e-30f;
    for (int base = blockIdx.x * 64; base < n; base += gridDim.x * 64) {
        const int i = base + lane;
        float ax = 0.f, ay = 0.f;
        if (i < n) {
            const float2 xi = xo[i];
            if (w == WAVES - 1) {  // the last wave holds the fewest packed words
                // neighbour votes in CSR order; loads batched four at a time;
                // high-degree rows were summed by k_heavy_edges
                const int e0 = rp[i], e1 = rp[i + 1];
                if (e1 - e0 > kHeavyDegree) {
                    const float2 hs = heavy_sum[heavy_index(heavy, nheavy, i)];
                    ax = hs.x;
                    ay = hs.y;
                }
                for (int e = e0; e1 - e0 <= kHeavyDegree && e < e1; e += 4) {
                    int j[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) j[q] = e + q < e1 ? ci[e + q] : i;
                    float2 xj[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) xj[q] = xo[j[q]];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float dx = xj[q].x - xi.x, dy = xj[q].y - xi.y;
                        float inv = __builtin_amdgcn_rsqf(dx * dx + (dy * dy + tiny));
                        float f = 1.f - inv;  // w = 1, d = 1
                        ax += f * dx;
                        ay += f * dy;
                    }
                }
            }
            if (w < nwords) {
                Packed<DT, VEC> nextw;
                nextw.v = dpk[(size_t)w * n + i];
                for (int b = w; b < nwords; b += WAVES) {
                    Packed<DT, VEC> u = nextw;
                    if (b + WAVES < nwords) nextw.v = dpk[(size_t)(b + WAVES) * n + i];  // prefetch
#pragma unroll
                    for (int jj = 0; jj < VEC; ++jj) {
                        const int t = b * VEC + jj;  // wave-uniform
                        const int d = (int)u.e[jj];
                        float f0, f1, hmul;          // f = hmul * (f0 - f1 * inv)
                        if (MODE == kHistLds) {
                            const int l = min(d >> 1, L - 1);
                            hmul = sH[t * L + l];
                            const float2 id = sTab[d];
                            f0 = id.x;
                            f1 = id.y;
                        } else {
                            const float2 e = MODE == kTableLds ? sTab[t * W + d] : wt2[(size_t)t * W + d];
                            f0 = e.x;
                            f1 = e.y;
                            hmul = 1.f;
                        }
                        const float2 p = sP[t];
                        float dx = p.x - xi.x, dy = p.y - xi.y;
                        float inv = __builtin_amdgcn_rsqf(dx * dx + (dy * dy + tiny));
                        float f = fmaf(-f1, inv, f0);
                        if (MODE == kHistLds) f *= hmul;
                        ax += f * dx;
                        ay += f * dy;
                    }
                }
            }
        }
        if (WAVES > 1) {
            sPart[w * 64 + lane] = make_float2(ax, ay);
            __syncthreads();
            if (w == 0) {
                for (int q = 1; q < WAVES; ++q) {
                    float2 o = sPart[q * 64 + lane];
                    ax += o.x;
                    ay += o.y;
                }
            }
        }
        if (w == 0 && i < n) {
            const float2 xi = xo[i];
            const float dn = den[i];
            xn[i] = make_float2(xi.x + ax / dn, xi.y + ay / dn);
        }
        if (WAVES > 1) __syncthreads();
    }
}

// ----------------------------------------------------------- stress

template <typename T2>
__device__ __forceinline__ double2 as_d2(const T2 v) {
    return make_double2((double)v.x, (double)v.y);
}

// Per-block partials of the sparse stress s'(x), Eq. 3, in FP64.
template <typename T2, typename DT, int VEC>
__global__ __launch_bounds__(256) void k_stress(int n, int kpad, int W, const int* __restrict__ rp,
                                                const int* __restrict__ ci, const T2* __restrict__ x,
                                                const uint4* __restrict__ dpk, const int* __restrict__ piv,
                                                const double* __restrict__ wt,
                                                double* __restrict__ partials) {
    extern __shared__ double2 sQ[];
    for (int t = threadIdx.x; t < kpad; t += blockDim.x) sQ[t] = as_d2(x[piv[t]]);
    __syncthreads();
    const int nwords = kpad / VEC;
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double2 xi = as_d2(x[i]);
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (j <= i) continue;
            double2 xj = as_d2(x[j]);
            double dx = xi.x - xj.x, dy = xi.y - xj.y;
            double r = sqrt(dx * dx + dy * dy);
            acc += (r - 1.0) * (r - 1.0);
        }
        for (int b = 0; b < nwords; ++b) {
            Packed<DT, VEC> u;
            u.v = dpk[(size_t)b * n + i];
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const int d = (int)u.e[j];
                if (d < 2) continue;
                const int t = b * VEC + j;
                const double2 p = sQ[t];
                double dx = xi.x - p.x, dy = xi.y - p.y;
                double r = sqrt(dx * dx + dy * dy);
                acc += wt[(size_t)t * W + d] * (r - d) * (r - d);
            }
        }
    }
    __shared__ double red[256 / kWave];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// Relative change of one sweep: partials of ||x_new - x_old||^2 and ||x_old||^2.
template <typename T2>
__global__ __launch_bounds__(256) void k_change(int n, const T2* __restrict__ xo, const T2* __restrict__ xn,
                                                double* __restrict__ partials) {
    double dd = 0.0, xx = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double2 a = as_d2(xo[i]), b = as_d2(xn[i]);
        dd += (b.x - a.x) * (b.x - a.x) + (b.y - a.y) * (b.y - a.y);
        xx += a.x * a.x + a.y * a.y;
    }
    __shared__ double red[256 / kWave];
    dd = block_sum(dd, red);
    xx = block_sum(xx, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = dd;
        partials[2 * blockIdx.x + 1] = xx;
    }
}

__global__ __launch_bounds__(256) void k_sum_pairs(const double* __restrict__ partials, int count,
                                                   double* __restrict__ out) {
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < count; q += blockDim.x) {
        a += partials[2 * q];
        b += partials[2 * q + 1];
    }
    __shared__ double red[256 / kWave];
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

// -------------------------------------------------------------- driver

struct SweepPlan {
    int grid = 1, block = 256, waves = 4, mode = kTableGlobal;
    size_t lds = 0;
};

template <typename DT, int VEC, int WAVES, int MODE>
static void launch_f32(const SweepPlan& pl, hipStream_t s, const ssm_csr* g, const ssm_terms* t,
                       const float2* xo, float2* xn) {
    hipLaunchKernelGGL((k_sweep_f32<DT, VEC, WAVES, MODE>), dim3(pl.grid), dim3(64 * WAVES), pl.lds, s, t->n,
                       t->kpad, t->W, t->delta_max + 1, g->row_ptr, g->col_idx, xo, xn, (const uint4*)t->dpk,
                       t->pivots, t->wt2, t->Hf, t->invd, t->den32, t->heavy, t->nheavy, t->heavy_sum);
}

template <typename DT, int VEC, int WAVES>
static void dispatch_mode(const SweepPlan& pl, hipStream_t s, const ssm_csr* g, const ssm_terms* t,
                          const float2* xo, float2* xn) {
    switch (pl.mode) {
        case kTableLds: launch_f32<DT, VEC, WAVES, kTableLds>(pl, s, g, t, xo, xn); break;
        case kHistLds: launch_f32<DT, VEC, WAVES, kHistLds>(pl, s, g, t, xo, xn); break;
        default: launch_f32<DT, VEC, WAVES, kTableGlobal>(pl, s, g, t, xo, xn); break;
    }
}

template <typename DT, int VEC>
static void dispatch_waves(const SweepPlan& pl, hipStream_t s, const ssm_csr* g, const ssm_terms* t,
                           const float2* xo, float2* xn) {
    switch (pl.waves) {
        case 1: dispatch_mode<DT, VEC, 1>(pl, s, g, t, xo, xn); break;
        case 2: dispatch_mode<DT, VEC, 2>(pl, s, g, t, xo, xn); break;
        case 4: dispatch_mode<DT, VEC, 4>(pl, s, g, t, xo, xn); break;
        default: dispatch_mode<DT, VEC, 8>(pl, s, g, t, xo, xn); break;
    }
}

static void sweep_once(const SweepPlan& pl, ssm_prec p, hipStream_t s, const ssm_csr* g, const ssm_terms* t,
                       const void* xo, void* xn) {
    if (p == SSM_FP64) {
        if (t->dbytes == 1)
            hipLaunchKernelGGL((k_sweep_f64<uint8_t, 16>), dim3(pl.grid), dim3(pl.block), pl.lds, s, t->n, t->kpad,
                               t->W, g->row_ptr, g->col_idx, (const double2*)xo, (double2*)xn,
                               (const uint4*)t->dpk, t->pivots, t->wtab64, t->den64);
        else
            hipLaunchKernelGGL((k_sweep_f64<uint16_t, 8>), dim3(pl.grid), dim3(pl.block), pl.lds, s, t->n, t->kpad,
                               t->W, g->row_ptr, g->col_idx, (const double2*)xo, (double2*)xn,
                               (const uint4*)t->dpk, t->pivots, t->wtab64, t->den64);
        return;
    }
    if (t->nheavy > 0)
        hipLaunchKernelGGL(k_heavy_edges, dim3(std::min(div_up(t->nheavy, 4), 4096)), dim3(256), 0, s, t->nheavy,
                           t->heavy, g->row_ptr, g->col_idx, (const float2*)xo, t->heavy_sum);
    if (t->dbytes == 1)
        dispatch_waves<uint8_t, 16>(pl, s, g, t, (const float2*)xo, (float2*)xn);
    else
        dispatch_waves<uint16_t, 8>(pl, s, g, t, (const float2*)xo, (float2*)xn);
}

static SweepPlan plan_sweep(const ssm_terms* t, ssm_prec p) {
    SweepPlan pl;
    const int nwords = t->kpad / t->vec;
    if (p == SSM_FP64) {
        pl.block = 256;
        pl.lds = sizeof(double) * 2 * (size_t)t->kpad;
        pl.grid = std::max(1, std::min(div_up(t->n, pl.block), num_cus() * 8));
        return pl;
    }
    // waves per 64-node chunk: aim at 8 resident waves per SIMD, never more
    // waves than packed words
    const long long chunks = div_up(t->n, 64);
    int waves = 1;
    while (waves < 4 && chunks * waves < 32LL * num_cus() && waves * 2 <= nwords) waves <<= 1;
    if (const char* v = getenv("SSM_SWEEP_WAVES")) {  // tuning override
        int f = atoi(v);
        if ((f == 1 || f == 2 || f == 4 || f == 8) && f <= nwords) waves = f;
    }
    pl.waves = waves;
    pl.block = 64 * waves;
    const size_t base = sizeof(float2) * ((size_t)t->kpad + 64 * (size_t)waves);
    const size_t table = sizeof(float2) * (size_t)t->kpad * t->W;
    const size_t hist = sizeof(float2) * (size_t)t->W + sizeof(float) * (size_t)t->kpad * (t->delta_max + 1);
    const size_t budget = 64 * 1024;
    if (base + table <= budget) {
        pl.mode = kTableLds;
        pl.lds = base + table;
    } else if (base + hist <= budget) {
        pl.mode = kHistLds;
        pl.lds = base + hist;
    } else {
        pl.mode = kTableGlobal;
        pl.lds = base;
    }
    // equal share of 64-node chunks per block; one chunk per block until the
    // LDS staging per block would matter (about 8 blocks per CU)
    long long max_grid = std::max<long long>(1, num_cus() * 8LL);
    if (const char* v = getenv("SSM_SWEEP_BLOCKS_PER_CU")) max_grid = std::max(1, atoi(v)) * (long long)num_cus();
    const long long per = (chunks + max_grid - 1) / max_grid;
    pl.grid = (int)std::max<long long>(1, (chunks + per - 1) / per);
    return pl;
}

ssm_status majorize(const ssm_csr* g, ssm_terms* t, ssm_prec p, void* x, int32_t iters, double tol,
                    int32_t* iters_done_host, hipStream_t s) {
    const SweepPlan pl = plan_sweep(t, p);
    const size_t xbytes = (p == SSM_FP64 ? sizeof(double) : sizeof(float)) * 2 * (size_t)t->n;
    void* bufs[2] = {x, t->xtmp};
    int cur = 0, done = 0;
    const int cblocks = std::min(div_up(t->n, 256), 2048);
    for (; done < iters; ++done) {
        sweep_once(pl, p, s, g, t, bufs[cur], bufs[cur ^ 1]);
        if (tol > 0.0) {
            if (p == SSM_FP64)
                hipLaunchKernelGGL(k_change<double2>, dim3(cblocks), dim3(256), 0, s, t->n,
                                   (const double2*)bufs[cur], (const double2*)bufs[cur ^ 1], t->red);
            else
                hipLaunchKernelGGL(k_change<float2>, dim3(cblocks), dim3(256), 0, s, t->n,
                                   (const float2*)bufs[cur], (const float2*)bufs[cur ^ 1], t->red);
            hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(256), 0, s, t->red, cblocks, t->red + 2 * cblocks);
            double h[2] = {0, 0};
            SSM_HIP(hipMemcpyAsync(h, t->red + 2 * cblocks, sizeof h, hipMemcpyDeviceToHost, s));
            SSM_HIP(hipStreamSynchronize(s));
            cur ^= 1;
            if (h[1] > 0.0 && sqrt(h[0]) / sqrt(h[1]) <= tol) {
                ++done;
                break;
            }
        } else {
            cur ^= 1;
        }
    }
    SSM_HIP(hipGetLastError());
    if (cur == 1) SSM_HIP(hipMemcpyAsync(x, t->xtmp, xbytes, hipMemcpyDeviceToDevice, s));
    if (iters_done_host) {
        SSM_HIP(hipStreamSynchronize(s));
        *iters_done_host = done;
    }
    return SSM_OK;
}

__global__ void k_round_layout(int n, const double2* __restrict__ a, float2* __restrict__ b) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double2 v = a[i];
        b[i] = make_float2((float)v.x, (float)v.y);
    }
}

ssm_status majorize_mixed(const ssm_csr* g, ssm_terms* t, double* x64, float* x32, int32_t iters, int32_t warm,
                          hipStream_t s) {
    const int first = std::min(iters, warm);
    ssm_status st = majorize(g, t, SSM_FP64, x64, first, 0.0, nullptr, s);
    if (st != SSM_OK) return st;
    hipLaunchKernelGGL(k_round_layout, dim3(std::min(div_up(t->n, 256), 4096)), dim3(256), 0, s, t->n,
                       (const double2*)x64, (float2*)x32);
    SSM_HIP(hipGetLastError());
    if (iters > first) return majorize(g, t, SSM_FP32, x32, iters - first, 0.0, nullptr, s);
    return SSM_OK;
}

ssm_status stress_sparse(const ssm_csr* g, ssm_terms* t, ssm_prec p, const void* x, double* out_host,
                         hipStream_t s) {
    const int blocks = std::min(div_up(t->n, 256), std::min(2048, t->red_len - 8));
    const size_t lds = sizeof(double) * 2 * (size_t)t->kpad;
    const uint4* dpk = (const uint4*)t->dpk;
    if (p == SSM_FP64) {
        if (t->dbytes == 1)
            hipLaunchKernelGGL((k_stress<double2, uint8_t, 16>), dim3(blocks), dim3(256), lds, s, t->n, t->kpad, t->W,
                               g->row_ptr, g->col_idx, (const double2*)x, dpk, t->pivots, t->wtab64, t->red);
        else
            hipLaunchKernelGGL((k_stress<double2, uint16_t, 8>), dim3(blocks), dim3(256), lds, s, t->n, t->kpad, t->W,
                               g->row_ptr, g->col_idx, (const double2*)x, dpk, t->pivots, t->wtab64, t->red);
    } else {
        if (t->dbytes == 1)
            hipLaunchKernelGGL((k_stress<float2, uint8_t, 16>), dim3(blocks), dim3(256), lds, s, t->n, t->kpad, t->W,
                               g->row_ptr, g->col_idx, (const float2*)x, dpk, t->pivots, t->wtab64, t->red);
        else
            hipLaunchKernelGGL((k_stress<float2, uint16_t, 8>), dim3(blocks), dim3(256), lds, s, t->n, t->kpad, t->W,
                               g->row_ptr, g->col_idx, (const float2*)x, dpk, t->pivots, t->wtab64, t->red);
    }
    launch_sum_partials(t->red, blocks, t->red + blocks, s);
    SSM_HIP(hipGetLastError());
    SSM_HIP(hipMemcpyAsync(out_host, t->red + blocks, sizeof(double), hipMemcpyDeviceToHost, s));
    SSM_HIP(hipStreamSynchronize(s));
    return SSM_OK;
}

// ------------------------------------------------------ full stress (Eq. 1)

// Sources s0 .. s0+nb-1 (BFS rows D): partials of sum over j > s of
// (r - d)^2 / d^2.
template <typename T2>
__global__ __launch_bounds__(256) void k_stress_full(int n, int s0, int nb, const int* __restrict__ D,
                                                     const T2* __restrict__ x, double* __restrict__ partials) {
    double acc = 0.0;
    long long total = (long long)nb * n;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        int r = (int)(q / n), j = (int)(q % n);
        int src = s0 + r;
        if (j <= src) continue;
        double d = (double)D[q];
        double2 a = as_d2(x[src]), b = as_d2(x[j]);
        double dx = a.x - b.x, dy = a.y - b.y;
        double dist = sqrt(dx * dx + dy * dy);
        acc += (dist - d) * (dist - d) / (d * d);
    }
    __shared__ double red[256 / kWave];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] += acc;
}

__global__ void k_iota(int* p, int s0, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = s0 + i;
}

ssm_status stress_full(const ssm_csr* g, ssm_prec p, const void* x, double* out_host, hipStream_t s) {
    const int n = g->n;
    const int nb = std::max(1, std::min(n, (1 << 26) / n));  // rows per batch (<= 256 MiB of distances)
    const int blocks = 1024;
    int* D = nullptr;
    int* src = nullptr;
    double* part = nullptr;
    ssm_status st = dalloc((void**)&D, sizeof(int) * (size_t)nb * n);
    if (st == SSM_OK) st = dalloc((void**)&src, sizeof(int) * (size_t)nb);
    if (st == SSM_OK) st = dalloc((void**)&part, sizeof(double) * (blocks + 1));
    if (st != SSM_OK) {
        if (D) hipFree(D);
        if (src) hipFree(src);
        return st;
    }
    hipError_t e = hipMemsetAsync(part, 0, sizeof(double) * (blocks + 1), s);
    for (int s0 = 0; s0 < n && e == hipSuccess && st == SSM_OK; s0 += nb) {
        int cnt = std::min(nb, n - s0);
        hipLaunchKernelGGL(k_iota, dim3(div_up(cnt, 256)), dim3(256), 0, s, src, s0, cnt);
        int32_t dm = 0;
        st = mssp(g, cnt, src, D, &dm, s);
        if (st != SSM_OK) break;
        if (p == SSM_FP64)
            hipLaunchKernelGGL(k_stress_full<double2>, dim3(blocks), dim3(256), 0, s, n, s0, cnt, D,
                               (const double2*)x, part);
        else
            hipLaunchKernelGGL(k_stress_full<float2>, dim3(blocks), dim3(256), 0, s, n, s0, cnt, D,
                               (const float2*)x, part);
        e = hipGetLastError();
    }
    if (st == SSM_OK && e == hipSuccess) {
        launch_sum_partials(part, blocks, part + blocks, s);
        e = hipMemcpyAsync(out_host, part + blocks, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    (void)hipFree(D);
    (void)hipFree(src);
    (void)hipFree(part);
    if (st != SSM_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "full stress");
    return SSM_OK;
}

}  // namespace ssm
