// Device code of the FP32 Jacobi sweep (paper Eq. 5): the packed-distance
// word type, the LDS staging helper, the heavy-row neighbour sums and the
// sweep kernel.  Host-side planning and launches live in sweep.hip.
#pragma once

#include "ssm_internal.h"
#include "wave.h"

namespace ssm {

template <typename DT, int VEC>
union Packed {
    uint4 v;
    DT e[VEC];
};

// --------------------------------------------------------- FP32 sweep

// A packed-distance word, read once per sweep.  With nt (a distance stream
// larger than half the MALL), a non-temporal load, so that the stream does
// not evict from L2 the coordinates that the neighbour gathers reuse
// (measured on MI355X: BA 146.8 -> 138.4 us, mesh 208 -> 197 us per sweep;
// a stream that stays in the MALL, 40 MB on the RGG, is slower with it).
__device__ __forceinline__ uint4 load_word(const uint4* p, bool nt) {
    if (!nt) return *p;
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    const v4u v = __builtin_nontemporal_load((const v4u*)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// How the FP32 sweep finds (w', w' d) for a pivot term.
enum WeightMode { kTableLds = 0, kHistLds = 1, kTableGlobal = 2 };

// Eq. 5 in displacement form: x_i' = x_i + (sum_q f_q (x_q - x_i)) / den_i
// with f_q = w_q - (w_q d_q) / r_iq, which equals num_i / den_i because every
// vote minus x_i is (x_q - x_i)(1 - d_q / r_iq).  Accumulating displacements
// keeps FP32 rounding relative to the (small) move rather than to the
// coordinates, and a vote at distance zero contributes exactly 0, so two
// coincident nodes with one closed neighbourhood get identical updates.
// 1/r is the hardware reciprocal square root of r^2 + 1e-30 (a zero
// displacement then still contributes exactly 0).

// Neighbour displacement sums of the heavy rows (degree > kHeavyDegree):
// one wavefront per segment of kHeavySeg arcs (lane l sums arcs l, l + 64,
// ... of the segment, then a fixed butterfly); the sweep adds a row's
// segments in order.  Same terms as the sweep's neighbour loop:
// (1 - 1/r) (x_j - x_i).
__global__ __launch_bounds__(256) void k_heavy_edges(int nseg, const int* __restrict__ heavy,
                                                     const int* __restrict__ seg_start,
                                                     const int* __restrict__ seg_owner, const int* __restrict__ rp,
                                                     const int* __restrict__ ci, const float2* __restrict__ xo,
                                                     float2* __restrict__ seg_sum, const int* __restrict__ stop) {
    if (stop[0]) return;  // the sweep loop has met its stop test
    const int lane = lane_id();
    const float tiny = 1e-30f;
    for (int q = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; q < nseg; q += gridDim.x * blockDim.x / kWave) {
        const int h = seg_owner[q];
        const int i = heavy[h];
        const int a = rp[i] + (q - seg_start[h]) * kHeavySeg;
        const int b = min(rp[i + 1], a + kHeavySeg);
        const float2 xi = xo[i];
        float ax = 0.f, ay = 0.f;
        for (int e = a + lane; e < b; e += kWave) {
            const float2 xj = xo[ci[e]];
            float dx = xj.x - xi.x, dy = xj.y - xi.y;
            float f = 1.f - __builtin_amdgcn_rsqf(dx * dx + (dy * dy + tiny));
            ax += f * dx;
            ay += f * dy;
        }
        ax = wave_sum(ax);
        ay = wave_sum(ay);
        if (lane == 0) seg_sum[q] = make_float2(ax, ay);
    }
}

// Copies nbytes (a multiple of 4) from global to LDS with 16-byte loads,
// four in flight per thread (both sides 16-byte aligned).  The loads are
// unconditional (an index past the end rereads the last word) so that they
// stay in registers and issue together; only the LDS stores are guarded.
__device__ __forceinline__ void stage_lds(void* dst, const void* __restrict__ src, size_t nbytes) {
    const int n16 = (int)(nbytes / 16);
    const int step = blockDim.x;
    uint4* d = (uint4*)dst;
    const uint4* g = (const uint4*)src;
    for (int q0 = threadIdx.x; q0 < n16; q0 += 4 * step) {
        const int last = n16 - 1;
        const uint4 v0 = g[q0];
        const uint4 v1 = g[min(q0 + step, last)];
        const uint4 v2 = g[min(q0 + 2 * step, last)];
        const uint4 v3 = g[min(q0 + 3 * step, last)];
        d[q0] = v0;
        if (q0 + step < n16) d[q0 + step] = v1;
        if (q0 + 2 * step < n16) d[q0 + 2 * step] = v2;
        if (q0 + 3 * step < n16) d[q0 + 3 * step] = v3;
    }
    for (int q = 4 * n16 + threadIdx.x; q < (int)(nbytes / 4); q += step)
        ((unsigned*)dst)[q] = ((const unsigned*)src)[q];
}

// Block = CPB groups of SPLIT wavefronts; a group takes 64 consecutive nodes
// (lane = node) and its SPLIT waves share the node's terms.  The terms are
// summed in four classes by packed-word index b mod 4, each class in
// ascending b (one coalesced 16-byte load per lane covers VEC pivots; two of
// a wave's words stay in flight); the neighbour terms, in CSR order (heavy
// rows: their segment sums in order), open class 3.  The node's sum is
// (A0 + A1) + (A2 + A3) whatever SPLIT is: wave s holds the classes
// congruent to s mod SPLIT, and wave 0 combines them (partials of the other
// waves through LDS).  So SPLIT, the block shape and the grid change the
// speed only, never a bit of the result.  Blocks loop over the chunks, so
// the LDS tables are staged once per block.
//
// Every lane of a wave reads the same pivot t, so the pivot's coordinates
// are wave-uniform loads from the contiguous array pc (kept current by the
// sweep itself: the node of pivot t writes its new coordinates into
// pc_next[t]).  The pivot term is f = w' - (w' d) / r: kTableLds stages
// (w', w' d) for every (pivot, distance) in LDS; kHistLds stages the region
// histograms H and (1/d^2, 1/d), w' = H[t][min(d/2, delta_max)] / d^2, so
// f = H (1/d^2 - (1/d) / r); kTableGlobal reads (w', w' d) from memory.
template <typename DT, int VEC, int SPLIT, int CPB, int MODE>
__global__ __launch_bounds__(64 * SPLIT * CPB) void k_sweep_f32(
    int n, int kpad, int W, int L, const int* __restrict__ rp, const int* __restrict__ ci,
    const float2* __restrict__ xo, float2* __restrict__ xn, const uint4* __restrict__ dpk,
    const float2* __restrict__ pc, float2* __restrict__ pc_next, const int* __restrict__ prank,
    const float2* __restrict__ wt2, const float* __restrict__ Hf, const float2* __restrict__ invd,
    const float* __restrict__ den, const int2* __restrict__ seg_range, const float2* __restrict__ seg_sum,
    const int* __restrict__ stop, bool nt) {
    if (stop[0]) return;  // the sweep loop has met its stop test (uniform over the grid)
    constexpr int NW = SPLIT * CPB;
    constexpr int R = 4 / SPLIT;  // classes per wave
    static_assert(SPLIT == 1 || SPLIT == 2 || SPLIT == 4, "waves per chunk");
    extern __shared__ float4 smem4[];
    float2* sP = (float2*)smem4;                                  // [kpad] pivot coordinates
    float2* sPart = sP + kpad;                                    // [2][NW][R][64] (SPLIT > 1)
    float2* sTab = sPart + (SPLIT > 1 ? 2 * NW * R * 64 : 0);     // kTableLds: [kpad][W]; kHistLds: invd [W]
    float* sH = (float*)(sTab + (MODE == kHistLds ? (W + 1) / 2 * 2 : 0));  // kHistLds: H [kpad][L]
    stage_lds(sP, pc, sizeof(float2) * (size_t)kpad);
    if (MODE == kTableLds) stage_lds(sTab, wt2, sizeof(float2) * (size_t)kpad * W);
    if (MODE == kHistLds) {
        stage_lds(sTab, invd, sizeof(float2) * (size_t)W);
        stage_lds(sH, Hf, sizeof(float) * (size_t)kpad * L);
    }
    __syncthreads();
    const int lane = threadIdx.x % 64;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);  // wave-uniform
    const int grp = w / SPLIT, sw = w % SPLIT;
    const int nwords = kpad / VEC;
    const int nchunks = (n + 63) / 64;
    const float tiny = 1e-30f;
    int buf = 0;
    for (int c0 = blockIdx.x * CPB; c0 < nchunks; c0 += gridDim.x * CPB) {  // uniform over the block
        const int i = (c0 + grp) * 64 + lane;
        float2 acc[R];
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = make_float2(0.f, 0.f);
        float2 xi = make_float2(0.f, 0.f);
        if (i < n) {
            xi = xo[i];
            Packed<DT, VEC> wa, wb;
            wa.v = sw < nwords ? load_word(&dpk[(size_t)sw * n + i], nt) : make_uint4(0, 0, 0, 0);
            wb.v = sw + SPLIT < nwords ? load_word(&dpk[(size_t)(sw + SPLIT) * n + i], nt) : make_uint4(0, 0, 0, 0);
            if (sw == SPLIT - 1) {  // the wave holding class 3
                float ax = 0.f, ay = 0.f;
                const int e0 = rp[i], e1 = rp[i + 1];
                if (e1 - e0 > kHeavyDegree) {  // the row's segment sums, in order
                    const int2 r = seg_range[i];
                    for (int q = r.x; q < r.y; ++q) {
                        const float2 hs = seg_sum[q];
                        ax += hs.x;
                        ay += hs.y;
                    }
                } else {
                    // neighbour votes in CSR order, eight gathers in flight
                    // (unconditional loads: a missing slot reads x_i itself)
                    for (int e = e0; e < e1; e += 8) {
                        int j[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int c = ci[min(e + q, e1 - 1)];  // unconditional load
                            j[q] = e + q < e1 ? c : i;
                        }
                        float2 xj[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) xj[q] = xo[j[q]];
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            // a missing slot holds x_i: zero displacement, adds exactly 0
                            float dx = xj[q].x - xi.x, dy = xj[q].y - xi.y;
                            float inv = __builtin_amdgcn_rsqf(dx * dx + (dy * dy + tiny));
                            float f = 1.f - inv;  // w = 1, d = 1
                            ax += f * dx;
                            ay += f * dy;
                        }
                    }
                }
                acc[R - 1] = make_float2(ax, ay);
            }
            // this wave's words b = sw, sw + SPLIT, ...: the j-th goes to class
            // (sw + j SPLIT) mod 4, local accumulator j mod R
            for (int b0 = sw; b0 < nwords; b0 += 4) {
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int b = b0 + q * SPLIT;
                    if (b >= nwords) break;
                    const Packed<DT, VEC> u = wa;
                    wa = wb;
                    if (b + 2 * SPLIT < nwords) wb.v = load_word(&dpk[(size_t)(b + 2 * SPLIT) * n + i], nt);  // two ahead
                    float ax = acc[q].x, ay = acc[q].y;
#pragma unroll
                    for (int jj = 0; jj < VEC; ++jj) {
                        const int t = b * VEC + jj;  // wave-uniform
                        const int d = (int)u.e[jj];
                        float f0, f1, hmul;  // f = hmul (f0 - f1 / r)
                        if (MODE == kHistLds) {
                            hmul = sH[t * L + min(d >> 1, L - 1)];
                            const float2 id = sTab[d];
                            f0 = id.x;
                            f1 = id.y;
                        } else {
                            const float2 e = MODE == kTableLds ? sTab[t * W + d] : wt2[(size_t)t * W + d];
                            f0 = e.x;
                            f1 = e.y;
                            hmul = 1.f;
                        }
                        const float2 p = sP[t];  // LDS broadcast
                        float dx = p.x - xi.x, dy = p.y - xi.y;
                        float inv = __builtin_amdgcn_rsqf(dx * dx + (dy * dy + tiny));
                        float f = fmaf(-f1, inv, f0);
                        if (MODE == kHistLds) f *= hmul;
                        ax += f * dx;
                        ay += f * dy;
                    }
                    acc[q] = make_float2(ax, ay);
                }
            }
        }
        float2 tot = make_float2(0.f, 0.f);
        if (SPLIT == 1) {
            tot = make_float2((acc[0].x + acc[1 % R].x) + (acc[2 % R].x + acc[3 % R].x),
                              (acc[0].y + acc[1 % R].y) + (acc[2 % R].y + acc[3 % R].y));
        } else {
            // partials double-buffered: one barrier per chunk group
#pragma unroll
            for (int q = 0; q < R; ++q) sPart[((buf * NW + w) * R + q) * 64 + lane] = acc[q];
            __syncthreads();
            if (sw == 0) {
                float2 A[4];  // class c lives in wave c mod SPLIT, local index c / SPLIT
#pragma unroll
                for (int c = 0; c < 4; ++c) A[c] = sPart[((buf * NW + w + c % SPLIT) * R + c / SPLIT) * 64 + lane];
                tot = make_float2((A[0].x + A[1].x) + (A[2].x + A[3].x), (A[0].y + A[1].y) + (A[2].y + A[3].y));
            }
            buf ^= 1;
        }
        if (sw == 0 && i < n) {
            const float dn = den[i];
            const float2 v = make_float2(xi.x + tot.x / dn, xi.y + tot.y / dn);
            xn[i] = v;
            const int r = prank[i];
            if (r >= 0) pc_next[r] = v;
        }
    }
}

}  // namespace ssm
