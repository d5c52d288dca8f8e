// Wavefront (64-lane) helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssm {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Rank of this lane among the set bits of `mask` below it.
__device__ __forceinline__ int mask_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Stream compaction: every active lane with `pred` gets a distinct slot from
// *tail; one atomic per wave (ballot + popcount + in-wave prefix).  Returns
// the slot, or -1 where pred is false.  Safe under divergence: the leader is
// the lowest active lane with pred set.
__device__ __forceinline__ int wave_append(bool pred, int* tail) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return -1;
    int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(tail, __popcll(mask));
    base = __shfl(base, leader);
    return pred ? base + mask_rank(mask) : -1;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Block-wide sum; every thread gets the result.  `scratch` holds one slot per
// wave.  Contains __syncthreads(); call from uniform control flow.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
    v = wave_sum(v);
    int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if (lane_id() == 0) scratch[w] = v;
    __syncthreads();
    T s = 0;
    for (int q = 0; q < nw; ++q) s += scratch[q];  // fixed order: deterministic
    return s;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T* scratch) {
    v = wave_max(v);
    int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if (lane_id() == 0) scratch[w] = v;
    __syncthreads();
    T s = scratch[0];
    for (int q = 1; q < nw; ++q) s = scratch[q] > s ? scratch[q] : s;
    return s;
}

// Calls f(i, j) for every arc (i, j) of the CSR rows i0 .. i0+63 (rows
// beyond n are empty): the wave walks the rows' arcs 64 at a time, so a
// long row costs its length / 64 passes instead of stalling one lane.  Lane
// l takes arcs e0 + l, e0 + l + 64, ... in that order, four per pass with
// their column loads in flight together.  Call with every lane of the wave
// active.
template <typename F>
__device__ __forceinline__ void wave_arcs(int n, const int* __restrict__ rp, const int* __restrict__ ci, int i0,
                                          F f) {
    constexpr int U = 4;
    const int lane = lane_id();
    const int end = rp[min(i0 + kWave, n)];
    const int a = i0 + lane < n ? rp[i0 + lane] : end;  // row start of this lane's node
    const int e0 = __shfl(a, 0);
    for (int eb = e0; eb < end; eb += U * kWave) {  // uniform
        int row[U], col[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = eb + u * kWave + lane;
            // the arc's row: the last lane whose row starts at or before e
            int lo = 0;
#pragma unroll
            for (int step = kWave / 2; step > 0; step >>= 1) {
                const int c = lo + step;
                if (__shfl(a, c) <= e) lo = c;
            }
            row[u] = i0 + lo;
            col[u] = e < end ? ci[e] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (eb + u * kWave + lane < end) f(row[u], col[u]);
    }
}

}  // namespace ssm
