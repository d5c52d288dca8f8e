// PivotMDS start layout and the rescale of Algorithm 1 (lines 3-4).
// The paper cites PivotMDS without defining it; the steps here follow the
// method it cites: double-centred squared pivot distances C (n x k), the
// Gram matrix C^T C (FP64 matrix cores), its two dominant eigenvectors by
// orthogonal iteration in FP64, and the projection x = C V.
#include <math.h>

#include <vector>

#include "ssm_internal.h"
#include "wave.h"

namespace ssm {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// colsum[t] = sum_i dist[t][i]^2 (exact in int64), from the packed copy:
// block b sums word row b (ranks b*VEC .. b*VEC+VEC-1).
template <typename DT, int VEC>
__global__ __launch_bounds__(256) void k_pmds_colsum(int n, int kpad, const uint4* __restrict__ dpk,
                                                     long long* __restrict__ colsum) {
    // block (b, y): packed word b over the y-th of gridDim.y node ranges;
    // partial sums colsum[y][rank] (exact integers, added up by k_pmds_mu)
    const int b = blockIdx.x;
    const int chunk = (n + gridDim.y - 1) / gridDim.y;
    const int i0 = blockIdx.y * chunk, i1 = min(n, i0 + chunk);
    long long s[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) s[j] = 0;
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        union {
            uint4 v;
            DT e[VEC];
        } u;
        u.v = dpk[(size_t)b * n + i];
#pragma unroll
        for (int j = 0; j < VEC; ++j) s[j] += (long long)u.e[j] * u.e[j];
    }
    __shared__ long long red[256 / kWave];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        long long tot = block_sum(s[j], red);
        if (threadIdx.x == 0) colsum[(size_t)blockIdx.y * kpad + b * VEC + j] = tot;
    }
}

// Node ranges of k_pmds_colsum per packed word.
constexpr int kColSplit = 32;

// mu[t] = colsum[t] / n with colsum[t] the sum of the kColSplit partials;
// stats[0] = gamma = sum_t colsum[t] / (n k).  Integer sums are exact, so
// these equal a serial double evaluation bit for bit.
__global__ void k_pmds_mu(int n, int k, int kpad, const long long* __restrict__ colsum, double* __restrict__ mu,
                          double* __restrict__ stats) {
    __shared__ long long tot[64];
    long long part = 0;
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        long long c = 0;
        for (int y = 0; y < kColSplit; ++y) c += colsum[(size_t)y * kpad + t];
        mu[t] = (double)c / (double)n;
        part += c;
    }
    tot[threadIdx.x] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long total = 0;
        for (int q = 0; q < (int)blockDim.x; ++q) total += tot[q];
        stats[0] = (double)total / ((double)n * (double)k);
    }
}

// nu[i] = sum_t dist[t][i]^2 / k (padding ranks hold 0 and add nothing).
template <typename DT, int VEC>
__global__ void k_pmds_nu(int n, int k, int nwords, const uint4* __restrict__ dpk, double* __restrict__ nu) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        long long s = 0;
        for (int b = 0; b < nwords; ++b) {
            union {
                uint4 v;
                DT e[VEC];
            } u;
            u.v = dpk[(size_t)b * n + i];
#pragma unroll
            for (int j = 0; j < VEC; ++j) s += (long long)u.e[j] * u.e[j];
        }
        nu[i] = (double)s / (double)k;
    }
}

__device__ __forceinline__ double centred(int d, double mu_t, double nu_i, double gamma) {
#pragma clang fp contract(off)
    double dd = (double)d;
    return -0.5 * (dd * dd - mu_t - nu_i + gamma);
}

// The same for a real distance d (graphs with edge lengths).
__device__ __forceinline__ double centred_d(double d, double mu_t, double nu_i, double gamma) {
#pragma clang fp contract(off)
    return -0.5 * (d * d - mu_t - nu_i + gamma);
}

constexpr int kGramTPW = 8;   // output tiles per wave
constexpr int kGramWaves = 4;
constexpr int kGramPF = 4;    // packed words per thread prefetched for the next round
#ifndef SSM_GRAM_PREFETCH
#define SSM_GRAM_PREFETCH 1
#endif
constexpr bool kGramPrefetch = SSM_GRAM_PREFETCH;
constexpr int kGramMinChunk = 256;  // nodes per Gram chunk at least

// Nodes staged per LDS round of the Gram product: 32 (eight K-steps of 4)
// when the staged block fits the default 64 KB of LDS, else 8.  The block
// holds C pivot-major, kp rows of SUB + 1 doubles (the odd stride keeps the
// staging stores of consecutive nodes in distinct banks), then mu.
template <int SUB>
constexpr size_t gram_lds_bytes(int kp) {
    return sizeof(double) * ((size_t)kp * (SUB + 1) + kp);
}
static int gram_sub(int kp) { return gram_lds_bytes<32>(kp) <= 64 * 1024 ? 32 : 8; }

// Split-K Gram product M = C^T C on v_mfma_f64_16x16x4_f64.  Block (c, g):
// node chunk c, tile group g (kGramWaves * kGramTPW tiles of the upper
// triangle).  C is formed on the fly from the packed distances and staged in
// LDS (SUB nodes per round); each wave accumulates its tiles over the chunk's
// nodes in ascending order and writes the chunk's partial tiles.  Operand
// layout per lane l: A[i][q] and B[q][j] with i = j = l % 16, q = l / 16;
// result lane l, element v holds row 4 v + l / 16, column l % 16.
template <typename DT, int VEC, int SUB>
__device__ __forceinline__ void pmds_gram_body(int c, int grp, int n, int k, int kp, int kpad, int chunk,
                                               const uint4* __restrict__ dpk, const double* __restrict__ mu,
                                               const double* __restrict__ nu, const double* __restrict__ stats,
                                               const int2* __restrict__ tiles, int ntiles,
                                               double* __restrict__ part) {
    constexpr int SP = SUB + 1;           // row stride of the staged block
    extern __shared__ double smem[];
    double* Cs = smem;                    // [kp][SP]: Cs[t * SP + r] = C of node i0 + r, pivot t
    double* smu = smem + (size_t)kp * SP; // [kp]
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    const double gamma = stats[0];
    for (int t = threadIdx.x; t < kp; t += blockDim.x) smu[t] = t < k ? mu[t] : 0.0;
    // this wave's tiles and their operand offsets in the staged block, read once
    int my_tiles[kGramTPW], offa[kGramTPW], offb[kGramTPW];
    int nmine = 0;
#pragma unroll
    for (int j = 0; j < kGramTPW; ++j) {
        const int id = (grp * kGramWaves + w) * kGramTPW + j;
        my_tiles[j] = id < ntiles ? id : -1;
        nmine += id < ntiles;
        const int2 ab = id < ntiles ? tiles[id] : make_int2(0, 0);
        offa[j] = 16 * ab.x * SP;
        offb[j] = 16 * ab.y * SP;
    }
    dbl4 acc[kGramTPW];
#pragma unroll
    for (int j = 0; j < kGramTPW; ++j) acc[j] = (dbl4){0.0, 0.0, 0.0, 0.0};
    const int i_begin = c * chunk, i_end = min(n, i_begin + chunk);
    const int nwords = VEC > 0 ? kpad / VEC : 0;
    // Packed inputs: when a round's SUB x nwords words fit kGramPF per thread,
    // the next round's words and nu are loaded into registers while this
    // round's MFMAs run.
    const bool pf = kGramPrefetch && VEC > 0 && SUB * nwords <= kGramPF * (int)blockDim.x;  // uniform
    uint4 pv[kGramPF];
    double pn[kGramPF];
    auto load_round = [&](int i0) {
#pragma unroll
        for (int p = 0; p < kGramPF; ++p) {
            const int q = threadIdx.x + p * (int)blockDim.x;
            const int r = q % SUB, i = i0 + r;
            const bool in = q < SUB * nwords && i < i_end;
            pv[p] = in ? dpk[(size_t)(q / SUB) * n + i] : make_uint4(0, 0, 0, 0);
            pn[p] = in ? nu[i] : 0.0;
        }
    };
    if (pf) load_round(i_begin);
    __syncthreads();
    for (int i0 = i_begin; i0 < i_end; i0 += SUB) {
        // stage C for nodes i0 .. i0 + SUB - 1 (zero past the chunk and past k);
        // VEC == 0: dpk holds real distance rows [k][n] (FP64)
        if constexpr (VEC == 0) {
            const double* dd = (const double*)dpk;
            for (int q = threadIdx.x; q < SUB * kp; q += blockDim.x) {
                const int r = q % SUB, t = q / SUB, i = i0 + r;
                Cs[t * SP + r] = (i < i_end && t < k) ? centred_d(dd[(size_t)t * n + i], smu[t], nu[i], gamma) : 0.0;
            }
        } else {
            auto put = [&](int q, const uint4 v, double nui) {  // the VEC values of item q
                const int r = q % SUB, b = q / SUB, i = i0 + r;
                union {
                    uint4 v;
                    DT e[VEC];
                } u;
                u.v = v;
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    const int t = b * VEC + j;
                    Cs[t * SP + r] = (i < i_end && t < k) ? centred((int)u.e[j], smu[t], nui, gamma) : 0.0;
                }
            };
            if (pf) {
#pragma unroll
                for (int p = 0; p < kGramPF; ++p) {
                    const int q = threadIdx.x + p * (int)blockDim.x;
                    if (q < SUB * nwords) put(q, pv[p], pn[p]);
                }
            } else {
                for (int q = threadIdx.x; q < SUB * nwords; q += blockDim.x) {
                    const int i = i0 + q % SUB;
                    put(q, i < i_end ? dpk[(size_t)(q / SUB) * n + i] : make_uint4(0, 0, 0, 0),
                        i < i_end ? nu[i] : 0.0);
                }
            }
            for (int q = threadIdx.x; q < SUB * (kp - kpad); q += blockDim.x) {
                const int r = q % SUB, t = kpad + q / SUB;
                Cs[t * SP + r] = 0.0;
            }
        }
        __syncthreads();
        if (pf && i0 + SUB < i_end) load_round(i0 + SUB);  // uniform
        const double* col = Cs + (lane % 16) * SP + lane / 16;
#pragma unroll
        for (int ks = 0; ks < SUB / 4; ++ks) {
#pragma unroll
            for (int j = 0; j < kGramTPW; ++j) {
                // a missing tile (j >= nmine) reads tile (0, 0) and is never stored
                const double a = col[offa[j] + 4 * ks];
                const double bb = col[offb[j] + 4 * ks];
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc[j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kGramTPW; ++j) {
        if (j < nmine) {
            double* out = part + ((size_t)c * ntiles + my_tiles[j]) * 256;
#pragma unroll
            for (int v = 0; v < 4; ++v) out[(4 * v + lane / 16) * 16 + (lane % 16)] = acc[j][v];
        }
    }
}

template <typename DT, int VEC, int SUB>
__global__ __launch_bounds__(256) void k_pmds_gram(int n, int k, int kp, int kpad, int chunk,
                                                   const uint4* __restrict__ dpk,
                                                   const double* __restrict__ mu,
                                                   const double* __restrict__ nu,
                                                   const double* __restrict__ stats,
                                                   const int2* __restrict__ tiles, int ntiles,
                                                   double* __restrict__ part) {
    pmds_gram_body<DT, VEC, SUB>(blockIdx.x, blockIdx.y, n, k, kp, kpad, chunk, dpk, mu, nu, stats, tiles, ntiles,
                                 part);
}

// Launches k_pmds_gram with the round size gram_sub(kp) (chunk a multiple of it).
template <typename DT, int VEC>
static void launch_gram(dim3 grid, hipStream_t s, int n, int k, int kp, int kpad, int chunk, const uint4* dpk,
                        const double* mu, const double* nu, const double* stats, const int2* tiles, int ntiles,
                        double* part) {
    if (gram_sub(kp) == 32) {
        hipLaunchKernelGGL((k_pmds_gram<DT, VEC, 32>), grid, dim3(256), gram_lds_bytes<32>(kp), s, n, k, kp, kpad,
                           chunk, dpk, mu, nu, stats, tiles, ntiles, part);
    } else {
        const size_t lds = gram_lds_bytes<8>(kp);
        if (lds > 64 * 1024)  // above the default dynamic LDS limit
            (void)hipFuncSetAttribute((const void*)k_pmds_gram<DT, VEC, 8>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_pmds_gram<DT, VEC, 8>), grid, dim3(256), lds, s, n, k, kp, kpad, chunk, dpk, mu, nu,
                           stats, tiles, ntiles, part);
    }
}

// M (k x k, row-major) = sum over chunks in ascending order of the partial
// tiles; the lower triangle mirrors the upper one.
__global__ void k_pmds_gram_reduce(int k, int nchunks, int ntiles, const int2* __restrict__ tiles,
                                   const double* __restrict__ part, double* __restrict__ M) {
    long long total = (long long)ntiles * 256;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        int tile = (int)(q / 256), e = (int)(q % 256);
        // chunks summed in ascending order, eight loads in flight
        const double* pp = part + (size_t)tile * 256 + e;
        const size_t stride = (size_t)ntiles * 256;
        double s = 0.0;
        int c = 0;
        for (; c + 8 <= nchunks; c += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = pp[(size_t)(c + u) * stride];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; c < nchunks; ++c) s += pp[(size_t)c * stride];
        int2 ab = tiles[tile];
        int r = 16 * ab.x + e / 16, col = 16 * ab.y + e % 16;
        if (r < k && col < k) {
            M[(size_t)r * k + col] = s;
            M[(size_t)col * k + r] = s;
        }
    }
}

__device__ __forceinline__ double splitmix_uniform(unsigned long long& state) {
    unsigned long long z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;  // [-1, 1)
}

constexpr int kEigP = 8;      // subspace width of the block iteration
constexpr int kEigThreads = 1024;  // the largest workgroup of the eigen kernels
// M in registers for k <= KR (KR = 128 or 256): KR / (waves) rows of M per
// wave, KR / 64 columns per lane.  KR = 128 runs on 512 threads, whose 256
// registers each hold the copy (at 1024 threads a thread has 128, and the
// copy spilled to scratch: a scratch round trip per row of M V); KR = 256
// runs on 512 threads too, with its rows below 128 in registers.
constexpr int kEigRegMax = 256;
__host__ __device__ constexpr int eig_threads(int KR) { return KR > 0 ? 512 : kEigThreads; }
// LDS bytes of pmds_eig_body for k.
__host__ __device__ constexpr size_t eig_lds_bytes(int k) {
    return sizeof(double) * ((size_t)(2 * kEigP + 2) * k + 2 * kEigP * kEigP + kEigP);
}
// Rows of M (from row 128 on) that the KR = 256 form keeps in LDS after
// pmds_eig_body's own arrays, within the workgroup's 160 KB (4 KB left for
// the static arrays).
constexpr long long kEigLdsBudget = 160 * 1024 - 4 * 1024;
__host__ __device__ constexpr int eig_m_lds_rows(int k) {
    return k <= 128 ? 0
                    : (int)(((long long)(k - 128) * k * 8 <= kEigLdsBudget - (long long)eig_lds_bytes(k))
                                ? (long long)(k - 128)
                                : (kEigLdsBudget - (long long)eig_lds_bytes(k)) / (8LL * k));
}
// Rows below 128 in registers; KR = 256 keeps its rows from 128 on in LDS as
// far as it holds them (eig_m_lds_rows) and reads the rest from memory.
__host__ __device__ constexpr int eig_reg_rows(int KR) {
    return KR > 0 ? (KR < 128 ? KR : 128) / (eig_threads(KR) / 64) : 1;
}
__host__ __device__ constexpr int eig_reg_cols(int KR) { return KR > 0 ? KR / 64 : 1; }
// The register form for a k x k Gram matrix: 128, 256, or 0 (M in global memory).
__host__ __device__ constexpr int eig_reg_form(int k) { return k <= 128 ? 128 : k <= kEigRegMax ? 256 : 0; }
// Steps of the two-vector iteration before the block iteration takes over.
// From step 32 on, every 16 steps, the residual's rate of decrease predicts
// the step at which it would converge; if that lies beyond kEigFast (or the
// residual stalls), the block iteration takes over at once: random trees
// with 5 % extra edges (lambda_3 / lambda_2 of 0.93-0.999) then take about
// 100 steps in all instead of 450, while meshes, grids and geometric graphs
// still converge within about 25 two-vector steps and power-law graphs
// within the budget (their block steps cost more at k = 200).
constexpr int kEigFast = 400;
constexpr int kEigProbe = 32;  // first step of the rate test
constexpr int kEigProbeEvery = 16;
constexpr int kEigCheck = 8;  // steps between Rayleigh-Ritz convergence tests

// Start / replacement vector entry (row r, column c, draw d): SplitMix64 in
// [-1, 1) from a state unique to (r, c, d).
__device__ __forceinline__ double eig_rand(int r, int c, int d) {
    unsigned long long st = 0x53534D00ull ^ ((unsigned long long)(unsigned)r << 20) ^
                            ((unsigned long long)c << 52) ^ ((unsigned long long)(unsigned)d << 56);
    return splitmix_uniform(st);
}

// Wave 0: orthonormalizes the first pw columns of A (k x kEigP, row-major,
// LDS) in place by classical Gram-Schmidt applied twice per column; a column
// whose remainder is negligible against the first column's norm (M of low
// rank) is replaced by a fresh random column.  Each lane owns rows lane,
// lane + 64, ...
__device__ void eig_orth(int k, int pw, double* A, int draw) {
    const int lane = lane_id();
    double ref = 0.0;
    for (int c = 0; c < pw; ++c) {
        for (int attempt = 0; attempt < 4; ++attempt) {
            for (int pass = 0; pass < 2; ++pass) {
                double d[kEigP];
#pragma unroll
                for (int b = 0; b < kEigP; ++b) d[b] = 0.0;
                for (int r = lane; r < k; r += kWave) {
                    const double ac = A[r * kEigP + c];
#pragma unroll
                    for (int b = 0; b < kEigP; ++b)
                        if (b < c) d[b] += A[r * kEigP + b] * ac;
                }
#pragma unroll
                for (int b = 0; b < kEigP; ++b)
                    if (b < c) d[b] = wave_sum_dpp(d[b]);
                for (int r = lane; r < k; r += kWave) {
                    double ac = A[r * kEigP + c];
#pragma unroll
                    for (int b = 0; b < kEigP; ++b)
                        if (b < c) ac -= d[b] * A[r * kEigP + b];
                    A[r * kEigP + c] = ac;
                }
            }
            double nn = 0.0;
            for (int r = lane; r < k; r += kWave) nn += A[r * kEigP + c] * A[r * kEigP + c];
            nn = sqrt(wave_sum_dpp(nn));
            if (c == 0 && attempt == 0) ref = nn > 0.0 ? nn : 1.0;
            if (nn > 1e-13 * ref) {
                for (int r = lane; r < k; r += kWave) A[r * kEigP + c] /= nn;
                break;
            }
            for (int r = lane; r < k; r += kWave) A[r * kEigP + c] = eig_rand(r, c, draw * 4 + attempt + 1);
        }
    }
}

// Eigen-decomposition of the symmetric leading pw x pw block of H
// (row-major, stride kEigP), one thread: cyclic Jacobi rotations until the
// off-diagonal part is below 1e-30 of the norm (or 64 sweeps).  Eigenvalues
// into th (descending), eigenvectors into the columns of Y in the same order.
// The working matrices live in LDS (ws: 2 kEigP^2 doubles): indexed by
// run-time rows and columns, as private arrays they went to scratch memory.
__device__ void eig_small(int pw, const double* H, double* Y, double* th, double* ws) {
    double(*a)[kEigP] = (double(*)[kEigP])ws;
    double(*v)[kEigP] = (double(*)[kEigP])(ws + kEigP * kEigP);
    for (int i = 0; i < kEigP; ++i)
        for (int j = 0; j < kEigP; ++j) {
            a[i][j] = i < pw && j < pw ? H[i * kEigP + j] : 0.0;
            v[i][j] = i == j ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < pw; ++i)
            for (int j = 0; j < pw; ++j) {
                tot += a[i][j] * a[i][j];
                if (i != j) off += a[i][j] * a[i][j];
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < pw - 1; ++p)
            for (int q = p + 1; q < pw; ++q) {
                if (a[p][q] == 0.0) continue;
                const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int r = 0; r < pw; ++r) {  // columns p, q
                    const double ap = a[r][p], aq = a[r][q];
                    a[r][p] = c * ap - sn * aq;
                    a[r][q] = sn * ap + c * aq;
                }
                for (int r = 0; r < pw; ++r) {  // rows p, q
                    const double ap = a[p][r], aq = a[q][r];
                    a[p][r] = c * ap - sn * aq;
                    a[q][r] = sn * ap + c * aq;
                }
                for (int r = 0; r < pw; ++r) {
                    const double vp = v[r][p], vq = v[r][q];
                    v[r][p] = c * vp - sn * vq;
                    v[r][q] = sn * vp + c * vq;
                }
            }
    }
    int order[kEigP];
    for (int i = 0; i < pw; ++i) order[i] = i;
    for (int i = 1; i < pw; ++i)  // insertion sort, descending (stable)
        for (int j = i; j > 0 && a[order[j]][order[j]] > a[order[j - 1]][order[j - 1]]; --j) {
            const int tmp = order[j];
            order[j] = order[j - 1];
            order[j - 1] = tmp;
        }
    for (int c = 0; c < kEigP; ++c) {
        th[c] = c < pw ? a[order[c]][order[c]] : 0.0;
        for (int r = 0; r < kEigP; ++r) Y[r * kEigP + c] = c < pw && r < pw ? v[r][order[c]] : 0.0;
    }
}

// The two dominant eigenvectors of the symmetric k x k matrix M, one
// workgroup: block subspace iteration on pw = min(kEigP, k) vectors (start:
// the SplitMix64 columns of eig_rand).  Each step: Z = M V (all waves), then
// V = an orthonormal basis of Z (wave 0).  Every kEigCheck steps V is
// replaced by its Rayleigh-Ritz basis (the pw x pw matrix V^T M V by cyclic
// Jacobi) and the two leading Ritz vectors U are tested: stop once every
// column of U lies in the span of the previous test's U to within `tol` per
// entry (only the first column when the second Ritz value is negligible, M
// of rank 1, or ties the third, where the second vector is not unique), or
// after max_iter steps.  The pair converges at the rate lambda_(pw+1) /
// lambda_2, so a near-tie of lambda_2 and lambda_3 costs nothing.  Then the
// sign rule: each column's largest-magnitude entry is positive (entries
// within a relative 1e-9 of the largest count as tied; the lowest index
// decides).  out: V (k x 2), lambda[2]; iters[0] = steps.
__device__ __forceinline__ void eigp_body(int k, const double* __restrict__ M, double tol, int max_iter,
                                          int steps0, double* __restrict__ out, int* __restrict__ iters) {
    extern __shared__ double sh[];
    double* V = sh;                  // [k][kEigP]
    double* Z = V + kEigP * k;       // [k][kEigP]
    double* U = Z + kEigP * k;       // [k][2] leading Ritz vectors of the last test
    double* H = U + 2 * k;           // [kEigP][kEigP]
    double* Y = H + kEigP * kEigP;   // [kEigP][kEigP]
    double* th = Y + kEigP * kEigP;  // [kEigP]
    __shared__ int s_done;
    __shared__ double red[kEigThreads / kWave];
    __shared__ double s_small[2 * kEigP * kEigP];  // eig_small's working matrices
    const int lane = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int pw = min(kEigP, k);
    for (int q = threadIdx.x; q < kEigP * k; q += blockDim.x) {
        const int r = q / kEigP, c = q % kEigP;
        V[q] = c < pw ? eig_rand(r, c, 0) : 0.0;
        Z[q] = 0.0;
    }
    for (int q = threadIdx.x; q < 2 * k; q += blockDim.x) U[q] = 0.0;
    if (threadIdx.x == 0) s_done = 0;
    __syncthreads();
    if (w == 0) eig_orth(k, pw, V, 0);
    __syncthreads();
    int it = 0;
    bool have_u = false;
    while (true) {
        // Z = M V: a wave per row, lanes over the columns of M
        for (int r = w; r < k; r += nw) {
            double acc[kEigP];
#pragma unroll
            for (int c = 0; c < kEigP; ++c) acc[c] = 0.0;
            for (int j = lane; j < k; j += kWave) {
                const double mv = M[(size_t)r * k + j];
#pragma unroll
                for (int c = 0; c < kEigP; ++c) acc[c] += mv * V[j * kEigP + c];
            }
#pragma unroll
            for (int c = 0; c < kEigP; ++c) acc[c] = wave_sum_dpp(acc[c]);
            if (lane < kEigP) {
                double mine = acc[0];
#pragma unroll
                for (int c = 1; c < kEigP; ++c)
                    if (lane == c) mine = acc[c];
                Z[r * kEigP + lane] = mine;
            }
        }
        ++it;
        __syncthreads();
        if (w == 0) {
            if (it % kEigCheck == 0 || it >= max_iter) {
                // Rayleigh-Ritz: H = V^T Z = V^T M V
                for (int a = 0; a < pw; ++a)
                    for (int b = a; b < pw; ++b) {
                        double d = 0.0;
                        for (int r = lane; r < k; r += kWave) d += V[r * kEigP + a] * Z[r * kEigP + b];
                        d = wave_sum_dpp(d);
                        if (lane == 0) {
                            H[a * kEigP + b] = d;
                            H[b * kEigP + a] = d;
                        }
                    }
                if (lane == 0) eig_small(pw, H, Y, th, s_small);
                __builtin_amdgcn_wave_barrier();
                const bool rank1 = !(fabs(th[1]) > 1e-13 * fabs(th[0]));
                const bool tie23 = pw > 2 && fabs(th[1] - th[2]) <= 1e-12 * fabs(th[0]);
                // U_new = V Y[:, 0:2], its distance from span(U_old); then
                // V = V Y (Ritz basis) and Z = Z Y (= M V Y)
                double p00 = 0.0, p01 = 0.0, p10 = 0.0, p11 = 0.0;
                for (int r = lane; r < k; r += kWave) {
                    double vr[kEigP], zr[kEigP];
#pragma unroll
                    for (int c = 0; c < kEigP; ++c) {
                        double v = 0.0, z = 0.0;
#pragma unroll
                        for (int b = 0; b < kEigP; ++b) {
                            v += V[r * kEigP + b] * Y[b * kEigP + c];
                            z += Z[r * kEigP + b] * Y[b * kEigP + c];
                        }
                        vr[c] = v;
                        zr[c] = z;
                    }
                    p00 += U[2 * r] * vr[0];
                    p01 += U[2 * r] * vr[1];
                    p10 += U[2 * r + 1] * vr[0];
                    p11 += U[2 * r + 1] * vr[1];
#pragma unroll
                    for (int c = 0; c < kEigP; ++c) {
                        V[r * kEigP + c] = vr[c];
                        Z[r * kEigP + c] = zr[c];
                    }
                }
                p00 = wave_sum_dpp(p00);
                p01 = wave_sum_dpp(p01);
                p10 = wave_sum_dpp(p10);
                p11 = wave_sum_dpp(p11);
                double res0 = 0.0, res1 = 0.0;
                for (int r = lane; r < k; r += kWave) {
                    const double u0 = V[r * kEigP + 0], u1 = V[r * kEigP + 1];
                    res0 = fmax(res0, fabs(u0 - p00 * U[2 * r] - p10 * U[2 * r + 1]));
                    res1 = fmax(res1, fabs(u1 - p01 * U[2 * r] - p11 * U[2 * r + 1]));
                    U[2 * r] = u0;
                    U[2 * r + 1] = u1;
                }
                res0 = wave_max_dpp(res0);
                res1 = wave_max_dpp(res1);
                const bool conv = have_u && res0 < tol && (res1 < tol || rank1 || tie23);
                if (lane == 0 && (conv || it >= max_iter)) s_done = 1;
                have_u = true;
            }
            // next basis: orthonormalized Z (= M V)
            for (int q = lane; q < kEigP * k; q += kWave) V[q] = Z[q];
            eig_orth(k, pw, V, it);
        }
        __syncthreads();
        if (s_done) break;  // uniform
    }
    // output: U (k x 2) with the sign rule, the Ritz values
    for (int col = 0; col < 2; ++col) {
        double mx = 0.0;
        for (int t = threadIdx.x; t < k; t += blockDim.x) mx = fmax(mx, fabs(U[2 * t + col]));
        mx = block_max(mx, red);
        int idx = k;  // lowest index within a relative 1e-9 of the largest magnitude
        for (int t = threadIdx.x; t < k; t += blockDim.x)
            if (fabs(U[2 * t + col]) >= mx * (1.0 - 1e-9) && t < idx) idx = t;
        idx = -block_max(-idx, (int*)red);
        if (idx >= k) idx = 0;
        const double sg = U[2 * idx + col] < 0.0 ? -1.0 : 1.0;
        for (int t = threadIdx.x; t < k; t += blockDim.x) out[2 * t + col] = sg * U[2 * t + col];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * k] = th[0];
        out[2 * k + 1] = th[1];
        iters[0] = steps0 + it;
    }
}

// Orthogonal (subspace) iteration on two vectors, one workgroup, M kept in
// registers when REG (k <= 256).  Start: SplitMix64 values in [-1, 1) (seed
// 0x53534D00 + column).  Each step: Z = M V, Gram-Schmidt; converged once
// every column of Z lies in span(V) to within `tol` per entry (only the first
// when M has numerical rank 1).  Then Rayleigh-Ritz on the 2 x 2 V^T M V
// (larger eigenvalue first) and the sign rule.  Returns false (uniformly,
// output untouched) when max_iter steps do not converge: the rate is
// lambda_3 / lambda_2, slow when those two nearly tie.
// N block-wide sums (or maxima) at once: each value is reduced exactly as
// block_sum (block_max) reduces one, with one pair of barriers for all N.
// scratch holds N slots per wave.
template <int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N], double* scratch) {
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int u = 0; u < N; ++u) v[u] = wave_sum_dpp(v[u]);
    __syncthreads();
    if (lane_id() == 0)
#pragma unroll
        for (int u = 0; u < N; ++u) scratch[u * nw + w] = v[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < N; ++u) {
        double t = 0;
        for (int q = 0; q < nw; ++q) t += scratch[u * nw + q];  // fixed order
        v[u] = t;
    }
}

template <int N>
__device__ __forceinline__ void block_max_n(double (&v)[N], double* scratch) {
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int u = 0; u < N; ++u) v[u] = wave_max_dpp(v[u]);
    __syncthreads();
    if (lane_id() == 0)
#pragma unroll
        for (int u = 0; u < N; ++u) scratch[u * nw + w] = v[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < N; ++u) {
        double t = scratch[u * nw];
        for (int q = 1; q < nw; ++q) t = scratch[u * nw + q] > t ? scratch[u * nw + q] : t;
        v[u] = t;
    }
}

template <int KR>
__device__ __forceinline__ bool eig2_body(int k, const double* __restrict__ M, double tol, int max_iter,
                                          double* __restrict__ out, int* __restrict__ iters, int& used, int mrows) {
    constexpr bool REG = KR > 0;
    constexpr int ER = eig_reg_rows(KR), EC = eig_reg_cols(KR);
    extern __shared__ double sh[];
    double* v0 = sh;
    double* v1 = sh + k;
    double* z0 = sh + 2 * k;
    double* z1 = sh + 3 * k;
    __shared__ double red[kEigThreads / kWave];
    __shared__ double red4[4 * (kEigThreads / kWave)];
    const int lane = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    double mreg[REG ? ER : 1][REG ? EC : 1];
    if (REG) {
#pragma unroll
        for (int q = 0; q < ER; ++q)
#pragma unroll
            for (int c = 0; c < EC; ++c) {
                int r = w + nw * q, j = lane + kWave * c;
                mreg[REG ? q : 0][REG ? c : 0] = (r < k && j < k) ? M[(size_t)r * k + j] : 0.0;
            }
    }
    // KR = 256: rows 128 .. 128 + mrows - 1 of M in LDS, after the iterations' own arrays
    double* Ml = sh + eig_lds_bytes(k) / sizeof(double);
    if (KR > 128)
        for (int q = threadIdx.x; q < mrows * k; q += blockDim.x) Ml[q] = M[(size_t)128 * k + q];
    if (threadIdx.x == 0) {
        unsigned long long s0 = 0x53534D00ull, s1 = 0x53534D01ull;
        for (int t = 0; t < k; ++t) {
            v0[t] = splitmix_uniform(s0);
            v1[t] = splitmix_uniform(s1);
        }
    }
    __syncthreads();
    // Shift of the REG iteration: Z = (M - sigma I) V (0 until set; see below)
    __shared__ double s_sigma;
    if (threadIdx.x == 0) s_sigma = 0.0;
    __syncthreads();
    auto matvec = [&]() {
        if (REG) {
            const double sigma = s_sigma;
            // this lane's entries of v0 and v1, read once (the z stores below
            // could otherwise force a reload per row)
            double x0[EC], x1[EC];
#pragma unroll
            for (int c = 0; c < EC; ++c) {
                const int j = lane + kWave * c;
                x0[c] = j < k ? v0[j] : 0.0;
                x1[c] = j < k ? v1[j] : 0.0;
            }
            // every row of the copy, also those beyond k (zero there, as are
            // x0 and x1 beyond k): no branch between the rows' sums, so
            // their lane moves interleave
#pragma unroll
            for (int q = 0; q < ER; ++q) {
                const int r = w + nw * q;
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int c = 0; c < EC; ++c) {
                    const double mv = mreg[REG ? q : 0][REG ? c : 0];
                    a0 += mv * x0[c];
                    a1 += mv * x1[c];
                }
                a0 = wave_sum_dpp(a0);
                a1 = wave_sum_dpp(a1);
                if (lane == 0 && r < k) {
                    z0[r] = sigma != 0.0 ? a0 - sigma * v0[r] : a0;
                    z1[r] = sigma != 0.0 ? a1 - sigma * v1[r] : a1;
                }
            }
            // KR = 256: the rows from 128 on, from LDS or memory, each lane's
            // columns in the same order as the register rows
            if (KR > 128) {
                for (int r = 128 + w; r < k; r += nw) {  // uniform across the wave
                    const double* row = r < 128 + mrows ? Ml + (size_t)(r - 128) * k : M + (size_t)r * k;
                    double a0 = 0.0, a1 = 0.0;
#pragma unroll
                    for (int c = 0; c < EC; ++c) {
                        const int j = lane + kWave * c;
                        const double mv = j < k ? row[j] : 0.0;
                        a0 += mv * x0[c];
                        a1 += mv * x1[c];
                    }
                    a0 = wave_sum_dpp(a0);
                    a1 = wave_sum_dpp(a1);
                    if (lane == 0) {
                        z0[r] = sigma != 0.0 ? a0 - sigma * v0[r] : a0;
                        z1[r] = sigma != 0.0 ? a1 - sigma * v1[r] : a1;
                    }
                }
            }
        } else {
            for (int r = w; r < k; r += nw) {
                double a0 = 0.0, a1 = 0.0;
                for (int j = lane; j < k; j += kWave) {
                    double mv = M[(size_t)r * k + j];
                    a0 += mv * v0[j];
                    a1 += mv * v1[j];
                }
                a0 = wave_sum_dpp(a0);
                a1 = wave_sum_dpp(a1);
                if (lane == 0) {
                    z0[r] = a0;
                    z1[r] = a1;
                }
            }
        }
        __syncthreads();
    };
    auto dot = [&](const double* a, const double* b) {
        double s = 0.0;
        for (int t = threadIdx.x; t < k; t += blockDim.x) s += a[t] * b[t];
        return block_sum(s, red);
    };
    int it = 0;
    bool converged = false;
    if constexpr (REG) {
        // k <= 256: the vector work of a step runs in wave 0 alone, entry
        // lane + 64 c of each vector in its registers (zero beyond k), sums
        // by shuffles; the other waves only join the product Z = M V.  A step
        // then costs two barriers instead of one pair per block-wide sum.
        constexpr int E = EC;
        __shared__ int s_flag;  // 0: go on, 1: converged, 2: the rate test hands over
        double vr0[E], vr1[E];
        auto wdot = [&](const double (&x)[E], const double (&y)[E]) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < E; ++c) acc += x[c] * y[c];
            return wave_sum_dpp(acc);
        };
        if (w == 0) {
#pragma unroll
            for (int c = 0; c < E; ++c) {
                const int t = lane + kWave * c;
                vr0[c] = t < k ? v0[t] : 0.0;
                vr1[c] = t < k ? v1[t] : 0.0;
            }
            // normalize v0, orthonormalize v1 against it (start vectors)
            const double nn = sqrt(wdot(vr0, vr0));
#pragma unroll
            for (int c = 0; c < E; ++c) vr0[c] /= nn;
            for (int pass = 0; pass < 2; ++pass) {
                const double d = wdot(vr0, vr1);
#pragma unroll
                for (int c = 0; c < E; ++c) vr1[c] -= d * vr0[c];
            }
            const double n1 = sqrt(wdot(vr1, vr1));
#pragma unroll
            for (int c = 0; c < E; ++c) {
                vr1[c] /= n1;
                const int t = lane + kWave * c;
                if (t < k) {
                    v0[t] = vr0[c];
                    v1[t] = vr1[c];
                }
            }
            if (lane == 0) s_flag = 0;
        }
        __syncthreads();
        double probe_res = -1.0;  // residual at step probe_it (rate test; wave 0)
        int probe_it = 0;
        bool shifted = false;     // wave 0: the shift has been chosen
        double sigma_next = 0.0;  // wave 0: the shift, published at the end of its step
        for (; it < max_iter; ++it) {
            matvec();
            if (w == 0) {
                double zr0[E], zr1[E];
#pragma unroll
                for (int c = 0; c < E; ++c) {
                    const int t = lane + kWave * c;
                    zr0[c] = t < k ? z0[t] : 0.0;
                    zr1[c] = t < k ? z1[t] : 0.0;
                }
                const double n0 = sqrt(wdot(zr0, zr0));
#pragma unroll
                for (int c = 0; c < E; ++c) zr0[c] /= n0;
                // Gram-Schmidt twice: once is not enough when z1 is nearly parallel to z0
                for (int pass = 0; pass < 2; ++pass) {
                    const double d01 = wdot(zr0, zr1);
#pragma unroll
                    for (int c = 0; c < E; ++c) zr1[c] -= d01 * zr0[c];
                }
                double n1 = sqrt(wdot(zr1, zr1));
                // a second column negligible against the first: M has numerical rank 1
                const bool rank1 = !(n1 > 1e-13 * n0);
                if (rank1) {
                    // any unit vector orthogonal to z0 will do: v1 made orthogonal to z0
#pragma unroll
                    for (int c = 0; c < E; ++c) zr1[c] = vr1[c];
                    for (int pass = 0; pass < 2; ++pass) {
                        const double d = wdot(zr0, zr1);
#pragma unroll
                        for (int c = 0; c < E; ++c) zr1[c] -= d * zr0[c];
                    }
                    n1 = sqrt(wdot(zr1, zr1));
                }
#pragma unroll
                for (int c = 0; c < E; ++c) zr1[c] /= n1;
                // distance of span(Z) from span(V): residual of projecting Z on V
                const double p00 = wdot(vr0, zr0), p10 = wdot(vr1, zr0);
                const double p01 = wdot(vr0, zr1), p11 = wdot(vr1, zr1);
                double res0 = 0.0, res1 = 0.0;
#pragma unroll
                for (int c = 0; c < E; ++c) {
                    res0 = fmax(res0, fabs(zr0[c] - p00 * vr0[c] - p10 * vr1[c]));
                    res1 = fmax(res1, fabs(zr1[c] - p01 * vr0[c] - p11 * vr1[c]));
                }
                res0 = wave_max_dpp(res0);
                res1 = wave_max_dpp(res1);
#pragma unroll
                for (int c = 0; c < E; ++c) {
                    vr0[c] = zr0[c];
                    vr1[c] = zr1[c];
                    const int t = lane + kWave * c;
                    if (t < k) {
                        v0[t] = zr0[c];
                        v1[t] = zr1[c];
                    }
                }
                int flag = 0;
                if (res0 < tol && (res1 < tol || rank1)) {
                    flag = 1;
                } else if (it + 1 >= kEigProbe && (it + 1 - kEigProbe) % kEigProbeEvery == 0) {
                    // rate test (values identical in every lane of wave 0)
                    const double r = fmax(res0, rank1 ? 0.0 : res1);
                    bool just_shifted = false;
                    if (probe_res > 0.0 && r > 0.0) {
                        double rate = pow(r / probe_res, 1.0 / (double)(it + 1 - probe_it));
                        // The span converges at the rate (l3 - s) / (l2 - s) of
                        // the shifted matrix.  M is a Gram matrix (its
                        // eigenvalues lie in [0, l3] below the top two), so
                        // s = l3 / 2 keeps the top two dominant and brings a
                        // slow rate q = l3 / l2 down to q / (2 - q): once,
                        // from the measured rate and the second column's
                        // norm (about l2), for rates above 1/2.
                        if (!shifted && rate > 0.5 && rate < 1.0 && !rank1 && n1 > 0.0) {
                            shifted = just_shifted = true;
                            const double l3 = rate * n1;
                            sigma_next = 0.5 * l3;
                            rate = rate / (2.0 - rate);
                        }
                        if (!(rate < 1.0) || (it + 1) + log(tol / r) / log(rate) > (double)max_iter) flag = 2;
                    }
                    // after the shift the next probe starts a new measurement
                    probe_res = just_shifted ? -1.0 : r;
                    probe_it = it + 1;
                }
                if (lane == 0) {
                    s_flag = flag;
                    if (flag == 0 && sigma_next != 0.0 && s_sigma == 0.0) s_sigma = sigma_next;
                }
            }
            __syncthreads();
            const int flag = s_flag;  // uniform
            if (flag == 1) {
                ++it;
                converged = true;
                break;
            }
            if (flag == 2) {
                ++it;  // this step is done
                break;
            }
        }
    } else {
        // normalize v0, orthonormalize v1 against it (start vectors)
        {
            double nn = sqrt(dot(v0, v0));
            for (int t = threadIdx.x; t < k; t += blockDim.x) v0[t] /= nn;
            __syncthreads();
            for (int pass = 0; pass < 2; ++pass) {
                double d = dot(v0, v1);
                for (int t = threadIdx.x; t < k; t += blockDim.x) v1[t] -= d * v0[t];
                __syncthreads();
            }
            double n1 = sqrt(dot(v1, v1));
            for (int t = threadIdx.x; t < k; t += blockDim.x) v1[t] /= n1;
            __syncthreads();
        }
        double probe_res = -1.0;  // residual at step probe_it (rate test)
        int probe_it = 0;
        for (; it < max_iter; ++it) {
            matvec();
            double n0 = sqrt(dot(z0, z0));
            for (int t = threadIdx.x; t < k; t += blockDim.x) z0[t] /= n0;
            __syncthreads();
            // Gram-Schmidt twice: once is not enough when z1 is nearly parallel to z0
            for (int pass = 0; pass < 2; ++pass) {
                double d01 = dot(z0, z1);
                for (int t = threadIdx.x; t < k; t += blockDim.x) z1[t] -= d01 * z0[t];
                __syncthreads();
            }
            double n1 = sqrt(dot(z1, z1));
            // a second column negligible against the first: M has numerical rank 1
            const bool rank1 = !(n1 > 1e-13 * n0);
            if (rank1) {
                // any unit vector orthogonal to z0 will do: keep v1 made orthogonal to z0
                for (int t = threadIdx.x; t < k; t += blockDim.x) z1[t] = v1[t];
                __syncthreads();
                for (int pass = 0; pass < 2; ++pass) {
                    double d = dot(z0, z1);
                    for (int t = threadIdx.x; t < k; t += blockDim.x) z1[t] -= d * z0[t];
                    __syncthreads();
                }
                n1 = sqrt(dot(z1, z1));
            }
            for (int t = threadIdx.x; t < k; t += blockDim.x) z1[t] /= n1;
            __syncthreads();
            // distance of span(Z) from span(V): residual of projecting Z on V
            // the four projections in one reduction, the two residuals in another
            double pr[4] = {0.0, 0.0, 0.0, 0.0};
            for (int t = threadIdx.x; t < k; t += blockDim.x) {
                pr[0] += v0[t] * z0[t];
                pr[1] += v1[t] * z0[t];
                pr[2] += v0[t] * z1[t];
                pr[3] += v1[t] * z1[t];
            }
            block_sum_n(pr, red4);
            const double p00 = pr[0], p10 = pr[1], p01 = pr[2], p11 = pr[3];
            double res[2] = {0.0, 0.0};
            for (int t = threadIdx.x; t < k; t += blockDim.x) {
                double r0 = z0[t] - p00 * v0[t] - p10 * v1[t];
                double r1 = z1[t] - p01 * v0[t] - p11 * v1[t];
                res[0] = fmax(res[0], fabs(r0));
                res[1] = fmax(res[1], fabs(r1));
            }
            block_max_n(res, red4);
            const double res0 = res[0], res1 = res[1];
            for (int t = threadIdx.x; t < k; t += blockDim.x) {
                v0[t] = z0[t];
                v1[t] = z1[t];
            }
            __syncthreads();
            if (res0 < tol && (res1 < tol || rank1)) {
                ++it;
                converged = true;
                break;
            }
            // rate test (values identical in every thread: uniform)
            if (it + 1 >= kEigProbe && (it + 1 - kEigProbe) % kEigProbeEvery == 0) {
                const double r = fmax(res0, rank1 ? 0.0 : res1);
                if (probe_res > 0.0 && r > 0.0) {
                    const double rate = pow(r / probe_res, 1.0 / (double)(it + 1 - probe_it));
                    if (!(rate < 1.0) || (it + 1) + log(tol / r) / log(rate) > (double)max_iter) {
                        ++it;  // this step is done
                        break;
                    }
                }
                probe_res = r;
                probe_it = it + 1;
            }
        }
    }
    used = it;
    if (!converged) return false;  // uniform: the caller goes on with the block iteration
    // Rayleigh-Ritz on span(V), with M itself
    if (threadIdx.x == 0) s_sigma = 0.0;
    __syncthreads();
    matvec();
    double b00 = dot(v0, z0), b11 = dot(v1, z1);
    double b01 = 0.5 * (dot(v0, z1) + dot(v1, z0));
    double th = 0.5 * atan2(2.0 * b01, b00 - b11);
    double cs = cos(th), sn = sin(th);
    double l0 = b00 * cs * cs + 2.0 * b01 * cs * sn + b11 * sn * sn;
    double l1 = b00 * sn * sn - 2.0 * b01 * cs * sn + b11 * cs * cs;
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        double a = v0[t], b = v1[t];
        z0[t] = cs * a + sn * b;
        z1[t] = -sn * a + cs * b;
    }
    __syncthreads();
    // sign rule
    for (int col = 0; col < 2; ++col) {
        double* z = col == 0 ? z0 : z1;
        double mx = 0.0;
        for (int t = threadIdx.x; t < k; t += blockDim.x) mx = fmax(mx, fabs(z[t]));
        mx = block_max(mx, red);
        int idx = k;  // lowest index within a relative 1e-9 of the largest magnitude
        for (int t = threadIdx.x; t < k; t += blockDim.x)
            if (fabs(z[t]) >= mx * (1.0 - 1e-9) && t < idx) idx = t;
        idx = -block_max(-idx, (int*)red);
        if (idx >= k) idx = 0;
        double sg = z[idx] < 0.0 ? -1.0 : 1.0;
        for (int t = threadIdx.x; t < k; t += blockDim.x) out[2 * t + col] = sg * z[t];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * k] = l0;
        out[2 * k + 1] = l1;
        iters[0] = it;
    }
    return true;
}

// The two dominant eigenvectors of M: the two-vector iteration for up to
// kEigFast steps (fewer when its rate test predicts it would not converge
// within them), then, if it has not converged, the block iteration.
template <int KR>
__device__ __forceinline__ void pmds_eig_body(int k, const double* __restrict__ M, double tol, int max_iter,
                                              double* __restrict__ out, int* __restrict__ iters, int mrows) {
    const int fast = min(max_iter, kEigFast);
    int used = 0;
    if (eig2_body<KR>(k, M, tol, fast, out, iters, used, mrows)) return;
    __syncthreads();
    eigp_body(k, M, tol, max_iter - used, used, out, iters);
}


template <int KR>
__global__ __launch_bounds__(eig_threads(KR)) void k_pmds_eig(int k, const double* __restrict__ M, double tol,
                                                         int max_iter, double* __restrict__ out,
                                                         int* __restrict__ iters, int mrows) {
    pmds_eig_body<KR>(k, M, tol, max_iter, out, iters, mrows);
}

// x_i = sum over t ascending of C_it V_t (per column), FP64.
template <typename DT, int VEC>
__global__ void k_pmds_project(int n, int k, int nwords, const uint4* __restrict__ dpk,
                               const double* __restrict__ mu, const double* __restrict__ nu,
                               const double* __restrict__ stats, const double* __restrict__ V,
                               double2* __restrict__ x) {
#pragma clang fp contract(off)
    const double gamma = stats[0];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s0 = 0.0, s1 = 0.0, nui = nu[i];
        for (int b = 0; b < nwords; ++b) {
            union {
                uint4 v;
                DT e[VEC];
            } u;
            u.v = dpk[(size_t)b * n + i];
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                int t = b * VEC + j;
                if (t < k) {
                    double c = centred((int)u.e[j], mu[t], nui, gamma);
                    s0 += c * V[2 * t];
                    s1 += c * V[2 * t + 1];
                }
            }
        }
        x[i] = make_double2(s0, s1);
    }
}

// Per-block partial sums of ||x_i - x_j|| over edges with j > i; every
// wave takes an equal share of the arcs (hub rows included).
__global__ __launch_bounds__(256) void k_pmds_edgelen(int n, const int* __restrict__ rp,
                                                      const int* __restrict__ ci,
                                                      const double2* __restrict__ x,
                                                      double* __restrict__ partials) {
    double s = 0.0;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int nwaves = gridDim.x * blockDim.x / kWave;
    const long long nnz = rp[n];
    wave_arc_span(n, rp, ci, (int)(nnz * wave / nwaves), (int)(nnz * (wave + 1) / nwaves), [&](int i, int j) {
        if (j <= i) return;
        const double2 xi = x[i], xj = x[j];
        double dx = xi.x - xj.x, dy = xi.y - xj.y;
        s += sqrt(dx * dx + dy * dy);
    });
    __shared__ double red[256 / kWave];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// x_out = c x with c = m / (summed edge lengths); flag[0] = 1 if that sum is 0.
template <typename T2>
__global__ void k_pmds_scale(int n, long long m, const double2* __restrict__ x, const double* __restrict__ have,
                             T2* __restrict__ out, int* flag) {
    const double h = have[0];
    if (h == 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) flag[0] = 1;
        return;
    }
    const double c = (double)m / h;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double2 v = x[i];
        out[i].x = v.x * c;
        out[i].y = v.y * c;
    }
}

ssm_status pivotmds(const ssm_csr* g, ssm_terms* t, ssm_prec p, void* x, hipStream_t s) {
    const int n = t->n, k = t->k;
    if (k > 1024) return fail(SSM_E_RANGE, "PivotMDS supports k <= 1024");
    const int kp = div_up(k, 16) * 16, T = kp / 16;
    std::vector<int2> htiles;
    for (int a = 0; a < T; ++a)
        for (int b = a; b < T; ++b) htiles.push_back(make_int2(a, b));
    const int ntiles = (int)htiles.size();
    const int per_group = kGramWaves * kGramTPW;
    const int ngroups = div_up(ntiles, per_group);
    int nchunks = std::max(1, std::min(div_up(n, kGramMinChunk), std::max(1, 4 * num_cus() / ngroups)));
    const int sub = gram_sub(kp);
    int chunk = div_up(div_up(n, nchunks), sub) * sub;
    nchunks = div_up(n, chunk);
    // workspace: colsum (k ll), mu (k), nu (n), stats (4), M (k*k), part, tiles, edge partials
    const int eblocks = std::min(div_up(n, 256), 2048);
    size_t bytes = sizeof(long long) * (size_t)kColSplit * t->kpad + sizeof(double) * ((size_t)k + n + 4) +
                   sizeof(double) * (size_t)nchunks * ntiles * 256 + sizeof(int2) * ntiles +
                   sizeof(double) * ((size_t)eblocks + 2) + 64 * 8;
    char* ws = nullptr;
    ssm_status st = salloc((void**)&ws, bytes);
    if (st != SSM_OK) return st;
    char* cur = ws;
    auto take = [&](size_t b) {
        char* r = cur;
        cur += (b + 63) / 64 * 64;
        return r;
    };
    long long* colsum = (long long*)take(sizeof(long long) * (size_t)kColSplit * t->kpad);
    double* mu = (double*)take(sizeof(double) * k);
    double* nu = (double*)take(sizeof(double) * n);
    double* stats = (double*)take(sizeof(double) * 4);
    double* M = t->gram;
    double* part = (double*)take(sizeof(double) * (size_t)nchunks * ntiles * 256);
    int2* tiles = (int2*)take(sizeof(int2) * ntiles);
    double* epart = (double*)take(sizeof(double) * ((size_t)eblocks + 2));
    int* flag = (int*)(epart + eblocks + 1);
    hipError_t e = hipMemcpyAsync(tiles, htiles.data(), sizeof(int2) * ntiles, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(flag, 0, sizeof(int), s);
    const int nwords = t->kpad / t->vec;
    const int gn = std::min(div_up(n, 256), 8192);
    const uint4* dpk = (const uint4*)t->dpk;
    if (e == hipSuccess) {
        if (t->dbytes == 1) {
            hipLaunchKernelGGL((k_pmds_colsum<uint8_t, 16>), dim3(nwords, kColSplit), dim3(256), 0, s, n, t->kpad, dpk,
                               colsum);
            hipLaunchKernelGGL((k_pmds_nu<uint8_t, 16>), dim3(gn), dim3(256), 0, s, n, k, nwords, dpk, nu);
        } else {
            hipLaunchKernelGGL((k_pmds_colsum<uint16_t, 8>), dim3(nwords, kColSplit), dim3(256), 0, s, n, t->kpad, dpk,
                               colsum);
            hipLaunchKernelGGL((k_pmds_nu<uint16_t, 8>), dim3(gn), dim3(256), 0, s, n, k, nwords, dpk, nu);
        }
        hipLaunchKernelGGL(k_pmds_mu, dim3(1), dim3(64), 0, s, n, k, t->kpad, colsum, mu, stats);
        dim3 gg(nchunks, ngroups);
        if (t->dbytes == 1)
            launch_gram<uint8_t, 16>(gg, s, n, k, kp, t->kpad, chunk, (const uint4*)t->dpk, mu, nu, stats, tiles,
                                     ntiles, part);
        else
            launch_gram<uint16_t, 8>(gg, s, n, k, kp, t->kpad, chunk, (const uint4*)t->dpk, mu, nu, stats, tiles,
                                     ntiles, part);
        hipLaunchKernelGGL(k_pmds_gram_reduce, dim3(std::min(div_up((long long)ntiles * 256, 256), 4096)),
                           dim3(256), 0, s, k, nchunks, ntiles, tiles, part, M);
        const size_t elds = eig_lds_bytes(k);
        if (eig_reg_form(k) == 128) {
            hipLaunchKernelGGL(k_pmds_eig<128>, dim3(1), dim3(eig_threads(128)), elds, s, k, M, 1e-13, 20000, t->eig,
                               t->eig_iters, 0);
        } else if (eig_reg_form(k) == 256) {
            const int mrows = eig_m_lds_rows(k);
            const size_t lds = elds + sizeof(double) * (size_t)mrows * k;
            if (lds > 64 * 1024)
                (void)hipFuncSetAttribute((const void*)k_pmds_eig<256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds);
            hipLaunchKernelGGL(k_pmds_eig<256>, dim3(1), dim3(eig_threads(256)), lds, s, k, M, 1e-13, 20000, t->eig,
                               t->eig_iters, mrows);
        } else {
            if (elds > 64 * 1024)
                (void)hipFuncSetAttribute((const void*)k_pmds_eig<0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)elds);
            hipLaunchKernelGGL(k_pmds_eig<0>, dim3(1), dim3(eig_threads(0)), elds, s, k, M, 1e-13, 20000, t->eig,
                               t->eig_iters, 0);
        }
        double2* xd = (double2*)t->xtmp;
        if (t->dbytes == 1)
            hipLaunchKernelGGL((k_pmds_project<uint8_t, 16>), dim3(gn), dim3(256), 0, s, n, k, nwords, dpk, mu,
                               nu, stats, t->eig, xd);
        else
            hipLaunchKernelGGL((k_pmds_project<uint16_t, 8>), dim3(gn), dim3(256), 0, s, n, k, nwords, dpk, mu,
                               nu, stats, t->eig, xd);
        hipLaunchKernelGGL(k_pmds_edgelen, dim3(eblocks), dim3(256), 0, s, n, g->row_ptr, g->col_idx, xd,
                           epart);
        launch_sum_partials(epart, eblocks, epart + eblocks, s);
        if (p == SSM_FP64)
            hipLaunchKernelGGL(k_pmds_scale<double2>, dim3(std::min(div_up(n, 256), 8192)), dim3(256), 0, s, n,
                               (long long)(g->nnz / 2), xd, epart + eblocks, (double2*)x, flag);
        else
            hipLaunchKernelGGL(k_pmds_scale<float2>, dim3(std::min(div_up(n, 256), 8192)), dim3(256), 0, s, n,
                               (long long)(g->nnz / 2), xd, epart + eblocks, (float2*)x, flag);
        e = hipGetLastError();
    }
    int hflag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);  // idle before the scratch is reused (also after an error)
    sfree(ws);
    if (e != hipSuccess) return hip_fail(e, "PivotMDS");
    if (hflag) return fail(SSM_E_INVAL, "PivotMDS layout has zero total edge length; cannot rescale");
    return SSM_OK;
}

// ------------------------------------------------------------ layout pool

// Per graph: colsum, mu, gamma and nu from its distance rows (the same exact
// integer sums and the same divisions as the single-graph path).
__global__ __launch_bounds__(1024) void k_pool_mds_stats(const PoolGraph* __restrict__ gs) {
    const PoolGraph& g = gs[blockIdx.x];
    const int n = g.n, k = g.k;
    __shared__ long long red[1024 / kWave];
    constexpr int U = 8;  // rows per pass (exact integer sums: any order)
    for (int t0 = 0; t0 < k; t0 += U) {
        long long s[U];
#pragma unroll
        for (int j = 0; j < U; ++j) s[j] = 0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            long long d[U];
#pragma unroll
            for (int j = 0; j < U; ++j) d[j] = t0 + j < k ? g.dist[(size_t)(t0 + j) * n + i] : 0;
#pragma unroll
            for (int j = 0; j < U; ++j) s[j] += d[j] * d[j];
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const long long v = block_sum(s[j], red);
            if (threadIdx.x == 0 && t0 + j < k) g.colsum[t0 + j] = v;
        }
    }
    if (threadIdx.x == 0) {  // colsum was written by this thread
        long long total = 0;
        for (int t = 0; t < k; ++t) {
            g.mu[t] = (double)g.colsum[t] / (double)n;
            total += g.colsum[t];
        }
        g.stats[0] = (double)total / ((double)n * (double)k);
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        long long s = 0;
        for (int t0 = 0; t0 < k; t0 += U) {
            long long d[U];
#pragma unroll
            for (int j = 0; j < U; ++j) d[j] = t0 + j < k ? g.dist[(size_t)(t0 + j) * n + i] : 0;
#pragma unroll
            for (int j = 0; j < U; ++j) s += d[j] * d[j];
        }
        g.nu[i] = (double)s / (double)k;
    }
}

// Items (graph, node chunk, tile group): the Gram partial tiles.
template <int SUB>
__global__ __launch_bounds__(256) void k_pool_gram(const PoolGraph* __restrict__ gs, const int4* __restrict__ items,
                                                   const int2* __restrict__ tiles) {
    const int4 it = items[blockIdx.x];
    const PoolGraph& g = gs[it.x];
    const int kp = (g.k + 15) / 16 * 16;
    pmds_gram_body<uint16_t, 8, SUB>(it.y, it.z, g.n, g.k, kp, g.kpad, kPoolGramChunk, g.dpk, g.mu, g.nu, g.stats,
                                     tiles, g.ntiles, g.gpart);
}

// Per graph (blockIdx.y): M = the chunks' partial tiles summed in ascending
// chunk order, mirrored into the lower triangle.
__global__ void k_pool_gram_reduce(const PoolGraph* __restrict__ gs, const int2* __restrict__ tiles) {
    const PoolGraph& g = gs[blockIdx.y];
    const long long total = (long long)g.ntiles * 256;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int tile = (int)(q / 256), e = (int)(q % 256);
        double s = 0.0;
        for (int c = 0; c < g.nchunks; ++c) s += g.gpart[((size_t)c * g.ntiles + tile) * 256 + e];
        const int2 ab = tiles[tile];
        const int r = 16 * ab.x + e / 16, col = 16 * ab.y + e % 16;
        if (r < g.k && col < g.k) {
            g.M[(size_t)r * g.k + col] = s;
            g.M[(size_t)col * g.k + r] = s;
        }
    }
}

template <int KR>
__global__ __launch_bounds__(eig_threads(KR)) void k_pool_eig(const PoolGraph* __restrict__ gs) {
    const PoolGraph& g = gs[blockIdx.x];
    pmds_eig_body<KR>(g.k, g.M, 1e-13, 20000, g.eig, g.info + 4, 0);
}

// Per graph: x64[0] = C V (ranks ascending), then the uniform rescale that
// makes the summed edge lengths equal m; info[3] = 1 if that sum is 0.
__global__ __launch_bounds__(1024) void k_pool_project(const PoolGraph* __restrict__ gs) {
#pragma clang fp contract(off)
    const PoolGraph& g = gs[blockIdx.x];
    const int n = g.n, k = g.k, nwords = g.kpad / 8;
    const double gamma = g.stats[0];
    double2* x = g.x64[0];
    // mu and the two eigenvectors in LDS (read by every node)
    __shared__ double s_mu[kPoolMaxK], s_v[2 * kPoolMaxK];
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        s_mu[t] = g.mu[t];
        s_v[2 * t] = g.eig[2 * t];
        s_v[2 * t + 1] = g.eig[2 * t + 1];
    }
    __syncthreads();
    constexpr int U = 4;  // packed words in flight per node
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double s0 = 0.0, s1 = 0.0;
        const double nui = g.nu[i];
        for (int b0 = 0; b0 < nwords; b0 += U) {
            union {
                uint4 v;
                uint16_t e[8];
            } u[U];
#pragma unroll
            for (int w = 0; w < U; ++w) u[w].v = b0 + w < nwords ? g.dpk[(size_t)(b0 + w) * n + i] : make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int w = 0; w < U; ++w) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int t = (b0 + w) * 8 + j;  // ranks in ascending order
                    if (t < k) {
                        const double c = centred((int)u[w].e[j], s_mu[t], nui, gamma);
                        s0 += c * s_v[2 * t];
                        s1 += c * s_v[2 * t + 1];
                    }
                }
            }
        }
        x[i] = make_double2(s0, s1);
    }
    __syncthreads();
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 xi = x[i];
        for (int e = g.rp[i]; e < g.rp[i + 1]; ++e) {
            const int j = g.ci[e];
            if (j <= i) continue;
            const double2 xj = x[j];
            const double dx = xi.x - xj.x, dy = xi.y - xj.y;
            s += sqrt(dx * dx + dy * dy);
        }
    }
    __shared__ double red[1024 / kWave];
    const double have = block_sum(s, red);
    if (have == 0.0) {
        if (threadIdx.x == 0) g.info[3] = 1;
        return;
    }
    const double c = (double)(g.nnz / 2) / have;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 v = x[i];
        x[i] = make_double2(v.x * c, v.y * c);
    }
}

hipError_t pool_pivotmds(const PoolGraph* gs, int count, const int4* gram_items, int ngram, const int2* tiles,
                         int kp_max, int k_max, hipStream_t s) {
    hipLaunchKernelGGL(k_pool_mds_stats, dim3(count), dim3(1024), 0, s, gs);
    // rounds of 32 nodes when the batch's largest staged block fits 64 KB (kPoolGramChunk is a multiple of 32)
    if (gram_sub(kp_max) == 32)
        hipLaunchKernelGGL(k_pool_gram<32>, dim3(ngram), dim3(256), gram_lds_bytes<32>(kp_max), s, gs, gram_items,
                           tiles);
    else
        hipLaunchKernelGGL(k_pool_gram<8>, dim3(ngram), dim3(256), gram_lds_bytes<8>(kp_max), s, gs, gram_items,
                           tiles);
    hipLaunchKernelGGL(k_pool_gram_reduce, dim3(32, count), dim3(256), 0, s, gs, tiles);
    if (eig_reg_form(k_max) == 128)
        hipLaunchKernelGGL(k_pool_eig<128>, dim3(count), dim3(eig_threads(128)), eig_lds_bytes(k_max), s, gs);
    else
        hipLaunchKernelGGL(k_pool_eig<256>, dim3(count), dim3(eig_threads(256)), eig_lds_bytes(k_max), s, gs);
    hipLaunchKernelGGL(k_pool_project, dim3(count), dim3(1024), 0, s, gs);
    return hipGetLastError();
}

// ------------------------------------------------- graphs with edge lengths

// colsum[t] = sum_i d_ti^2 for real distances (block t).
__global__ __launch_bounds__(256) void k_wpmds_colsum(int n, const double* __restrict__ dist,
                                                      double* __restrict__ colsum) {
    const int t = blockIdx.x;
    double s = 0.0;
    const int B = blockDim.x;
    for (int i0 = threadIdx.x; i0 < n; i0 += 4 * B) {
        double d[4];  // four loads in flight, added in the same order as one at a time
#pragma unroll
        for (int j = 0; j < 4; ++j) d[j] = i0 + j * B < n ? dist[(size_t)t * n + i0 + j * B] : 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (i0 + j * B < n) s += d[j] * d[j];
    }
    __shared__ double red[256 / kWave];
    s = block_sum(s, red);
    if (threadIdx.x == 0) colsum[t] = s;
}

__global__ void k_wpmds_mu(int n, int k, const double* __restrict__ colsum, double* __restrict__ mu,
                           double* __restrict__ stats) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double total = 0.0;
        for (int t = 0; t < k; ++t) {
            mu[t] = colsum[t] / (double)n;
            total += colsum[t];
        }
        stats[0] = total / ((double)n * (double)k);
    }
}

__global__ void k_wpmds_nu(int n, int k, const double* __restrict__ dist, double* __restrict__ nu) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        constexpr int U = 8;  // loads in flight; the sum keeps ascending ranks
        for (int t0 = 0; t0 < k; t0 += U) {
            double dv[U];
#pragma unroll
            for (int j = 0; j < U; ++j) dv[j] = t0 + j < k ? dist[(size_t)(t0 + j) * n + i] : 0.0;
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (t0 + j < k) s += dv[j] * dv[j];
        }
        nu[i] = s / (double)k;
    }
}

__global__ void k_wpmds_project(int n, int k, const double* __restrict__ dist, const double* __restrict__ mu,
                                const double* __restrict__ nu, const double* __restrict__ stats,
                                const double* __restrict__ V, double2* __restrict__ x) {
#pragma clang fp contract(off)
    const double gamma = stats[0];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s0 = 0.0, s1 = 0.0;
        const double nui = nu[i];
        for (int t = 0; t < k; ++t) {
            const double c = centred_d(dist[(size_t)t * n + i], mu[t], nui, gamma);
            s0 += c * V[2 * t];
            s1 += c * V[2 * t + 1];
        }
        x[i] = make_double2(s0, s1);
    }
}

// Per-block partials of the drawn edge lengths and of the edge lengths
// (edges j > i): partials[b] and partials[nb + b].
__global__ __launch_bounds__(256) void k_wpmds_edgelen(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ len, const double2* __restrict__ x,
                                                       double* __restrict__ partials) {
    double have = 0.0, target = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double2 xi = x[i];
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int j = ci[e];
            if (j <= i) continue;
            const double2 xj = x[j];
            const double dx = xi.x - xj.x, dy = xi.y - xj.y;
            have += sqrt(dx * dx + dy * dy);
            target += len[e];
        }
    }
    __shared__ double red[256 / kWave];
    have = block_sum(have, red);
    target = block_sum(target, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = have;
        partials[gridDim.x + blockIdx.x] = target;
    }
}

// x_out = c x, c = (summed lengths) / (summed drawn lengths); flag if that is 0.
template <typename T2>
__global__ void k_wpmds_scale(int n, const double2* __restrict__ x, const double* __restrict__ sums,
                              T2* __restrict__ out, int* flag) {
    const double have = sums[0], target = sums[1];
    if (have == 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) flag[0] = 1;
        return;
    }
    const double c = target / have;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double2 v = x[i];
        out[i].x = v.x * c;
        out[i].y = v.y * c;
    }
}

// sums[0], sums[1] = the two partial arrays summed in block order.
// sums[0..1] = the two rows of partials [2][nb] summed by one wave: lane l
// adds q = l, l + 64, ... in ascending order, then a fixed-order wave sum
// (deterministic).
__global__ void k_wpmds_sum2(int nb, const double* __restrict__ partials, double* __restrict__ sums) {
    if (blockIdx.x != 0 || threadIdx.x >= kWave) return;
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < nb; q += kWave) {
        a += partials[q];
        b += partials[nb + q];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (threadIdx.x == 0) {
        sums[0] = a;
        sums[1] = b;
    }
}

ssm_status pivotmds_w(const ssm_csr* g, const double* len, int k, const double* dist, ssm_prec p, void* x,
                      hipStream_t s) {
    const int n = g->n;
    if (k > 1024) return fail(SSM_E_RANGE, "PivotMDS supports k <= 1024");
    const int kp = div_up(k, 16) * 16, T = kp / 16;
    std::vector<int2> htiles;
    for (int a = 0; a < T; ++a)
        for (int b = a; b < T; ++b) htiles.push_back(make_int2(a, b));
    const int ntiles = (int)htiles.size();
    const int ngroups = div_up(ntiles, kGramWaves * kGramTPW);
    int nchunks = std::max(1, std::min(div_up(n, kGramMinChunk), std::max(1, 4 * num_cus() / ngroups)));
    const int sub = gram_sub(kp);
    const int chunk = div_up(div_up(n, nchunks), sub) * sub;
    nchunks = div_up(n, chunk);
    const int eb = std::min(div_up(n, 256), 2048);
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += (b + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_cs = take(sizeof(double) * k), o_mu = take(sizeof(double) * k), o_nu = take(sizeof(double) * n),
                 o_st = take(sizeof(double) * 4), o_M = take(sizeof(double) * (size_t)k * k),
                 o_part = take(sizeof(double) * (size_t)nchunks * ntiles * 256), o_tiles = take(sizeof(int2) * ntiles),
                 o_eig = take(sizeof(double) * (2 * (size_t)k + 2)), o_it = take(sizeof(int) * 2),
                 o_x = take(sizeof(double2) * n), o_ep = take(sizeof(double) * 2 * (size_t)eb),
                 o_sums = take(sizeof(double) * 2);
    char* ws = nullptr;
    ssm_status st = salloc((void**)&ws, off);
    if (st != SSM_OK) return st;
    double* colsum = (double*)(ws + o_cs);
    double* mu = (double*)(ws + o_mu);
    double* nu = (double*)(ws + o_nu);
    double* stats = (double*)(ws + o_st);
    double* M = (double*)(ws + o_M);
    double* part = (double*)(ws + o_part);
    int2* tiles = (int2*)(ws + o_tiles);
    double* eig = (double*)(ws + o_eig);
    int* its = (int*)(ws + o_it);
    int* flag = its + 1;
    double2* xd = (double2*)(ws + o_x);
    double* epart = (double*)(ws + o_ep);
    double* sums = (double*)(ws + o_sums);
    hipError_t e = hipMemcpyAsync(tiles, htiles.data(), sizeof(int2) * ntiles, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(its, 0, sizeof(int) * 2, s);
    if (e == hipSuccess) {
        const int gn = std::min(div_up(n, 256), 8192);
        hipLaunchKernelGGL(k_wpmds_colsum, dim3(k), dim3(256), 0, s, n, dist, colsum);
        hipLaunchKernelGGL(k_wpmds_mu, dim3(1), dim3(64), 0, s, n, k, colsum, mu, stats);
        hipLaunchKernelGGL(k_wpmds_nu, dim3(gn), dim3(256), 0, s, n, k, dist, nu);
        launch_gram<double, 0>(dim3(nchunks, ngroups), s, n, k, kp, kp, chunk, (const uint4*)dist, mu, nu, stats,
                               tiles, ntiles, part);
        hipLaunchKernelGGL(k_pmds_gram_reduce, dim3(std::min(div_up((long long)ntiles * 256, 256), 4096)), dim3(256),
                           0, s, k, nchunks, ntiles, tiles, part, M);
        const size_t elds = eig_lds_bytes(k);
        if (eig_reg_form(k) == 128) {
            hipLaunchKernelGGL(k_pmds_eig<128>, dim3(1), dim3(eig_threads(128)), elds, s, k, M, 1e-13, 20000, eig, its,
                               0);
        } else if (eig_reg_form(k) == 256) {
            const int mrows = eig_m_lds_rows(k);
            const size_t lds = elds + sizeof(double) * (size_t)mrows * k;
            if (lds > 64 * 1024)
                (void)hipFuncSetAttribute((const void*)k_pmds_eig<256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds);
            hipLaunchKernelGGL(k_pmds_eig<256>, dim3(1), dim3(eig_threads(256)), lds, s, k, M, 1e-13, 20000, eig, its,
                               mrows);
        } else {
            if (elds > 64 * 1024)
                (void)hipFuncSetAttribute((const void*)k_pmds_eig<0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)elds);
            hipLaunchKernelGGL(k_pmds_eig<0>, dim3(1), dim3(eig_threads(0)), elds, s, k, M, 1e-13, 20000, eig, its, 0);
        }
        hipLaunchKernelGGL(k_wpmds_project, dim3(gn), dim3(256), 0, s, n, k, dist, mu, nu, stats, eig, xd);
        hipLaunchKernelGGL(k_wpmds_edgelen, dim3(eb), dim3(256), 0, s, n, g->row_ptr, g->col_idx, len, xd, epart);
        hipLaunchKernelGGL(k_wpmds_sum2, dim3(1), dim3(64), 0, s, eb, epart, sums);
        if (p == SSM_FP64)
            hipLaunchKernelGGL(k_wpmds_scale<double2>, dim3(gn), dim3(256), 0, s, n, xd, sums, (double2*)x, flag);
        else
            hipLaunchKernelGGL(k_wpmds_scale<float2>, dim3(gn), dim3(256), 0, s, n, xd, sums, (float2*)x, flag);
        e = hipGetLastError();
    }
    int hflag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    sfree(ws);
    if (e != hipSuccess) return hip_fail(e, "PivotMDS (edge lengths)");
    if (hflag) return fail(SSM_E_INVAL, "PivotMDS layout has zero total edge length; cannot rescale");
    return SSM_OK;
}

}  // namespace ssm
