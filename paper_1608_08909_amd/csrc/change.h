// Algorithm 1's stop test on the device: the relative positional change of
// one sweep after the best proper rigid motion (rotation and translation) of
// the old layout onto the new one, relative to the old layout's spread about
// its centroid.  Computed from twelve first and second moments of the old
// and new coordinates, both taken relative to one reference point o (a node
// of the old layout, which keeps the moments' cancellation small); the
// moments are summed in FP64 in a fixed order for a given launch shape.
#pragma once

#include <math.h>

#include "ssm_internal.h"
#include "wave.h"

namespace ssm {

constexpr int kMoments = 12;

// m: sum a, sum b (2 each), sum a.a, b.b componentwise (2 each), then the
// four cross sums a.x b.x, a.x b.y, a.y b.x, a.y b.y, with a = x_old - o and
// b = x_new - o.
__device__ __forceinline__ void moments_add(double (&m)[kMoments], double2 o, double2 xo, double2 xn) {
    const double ax = xo.x - o.x, ay = xo.y - o.y, bx = xn.x - o.x, by = xn.y - o.y;
    m[0] += ax;
    m[1] += ay;
    m[2] += bx;
    m[3] += by;
    m[4] += ax * ax;
    m[5] += ay * ay;
    m[6] += bx * bx;
    m[7] += by * by;
    m[8] += ax * bx;
    m[9] += ax * by;
    m[10] += ay * bx;
    m[11] += ay * by;
}

// The change from the summed moments of n nodes: with centred a, b, the
// spread aa = sum |a|^2, bb = sum |b|^2, P = sum a.b, Q = sum (a.x b.y -
// a.y b.x); the best rotation leaves aa + bb - 2 sqrt(P^2 + Q^2).  +infinity
// when the old layout has no spread.
__device__ __forceinline__ double rigid_change(const double (&m)[kMoments], int n) {
    const double dn = (double)n;
    const double mx = m[0] / dn, my = m[1] / dn, nx = m[2] / dn, ny = m[3] / dn;
    const double aa = (m[4] - dn * mx * mx) + (m[5] - dn * my * my);
    const double bb = (m[6] - dn * nx * nx) + (m[7] - dn * ny * ny);
    const double P = (m[8] - dn * mx * nx) + (m[11] - dn * my * ny);
    const double Q = (m[9] - dn * mx * ny) - (m[10] - dn * my * nx);
    if (!(aa > 0.0)) return INFINITY;
    const double res = aa + bb - 2.0 * sqrt(P * P + Q * Q);
    return sqrt(fmax(res, 0.0) / aa);
}

template <typename T2>
__device__ __forceinline__ double2 to_d2(const T2 v) {
    return make_double2((double)v.x, (double)v.y);
}

// The twelve moments summed over a 256-thread block: wave sums by DPP, one
// barrier, then a fixed-order sum over the waves; thread j < kMoments gets
// moment j.  Call from uniform control flow.
__device__ __forceinline__ double block_moments(const double (&m)[kMoments], double* red) {
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < kMoments; ++j) {
        const double v = wave_sum_dpp(m[j]);
        if (lane_id() == 0) red[w * kMoments + j] = v;
    }
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < kMoments)
        for (int q = 0; q < 256 / kWave; ++q) t += red[q * kMoments + threadIdx.x];
    return t;
}

}  // namespace ssm
