/*
 * ssm_oracle.c - plain, slow, serial FP64 CPU oracle of the sparse stress
 * model (Ortmann, Klimenta, Brandes: "A Sparse Stress Model", Section 3,
 * Algorithm 1, Eqs. 1, 3, 5), for unit edge lengths and, at the end of the
 * file, for Algorithm 1's general input with positive edge lengths.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  It shares no code, header,
 * table or helper with the GPU library and includes nothing from it.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 * Every floating-point step is IEEE double with correctly rounded sqrt and
 * division; sums run in the order stated beside each function.
 *
 * Readings of the paper where it is silent or ambiguous (each is listed in the
 * design notes as well):
 *   - Update order: Jacobi (every node reads the previous iterate); the
 *     in-place order that Algorithm 1 writes is kept as an option only.
 *   - The second sum of the update's denominator is over w'_ip (the paper
 *     prints w'_ij there).
 *   - A pivot term (i, p) exists iff d_ip >= 2: it excludes p = i (w'_ii would
 *     divide by zero) and p in N(i) (as Eq. 3 states).
 *   - d_jp <= d_ip / 2 is read over the reals, i.e. delta_j <= floor(d_ip/2).
 *   - Region ties (Section 3: the currently smallest partition wins) are
 *     resolved level by level: at distance l, nodes with one nearest pivot
 *     join it first; then all tied nodes at l pick, against a snapshot of the
 *     sizes, the candidate with the smallest (size, pivot rank).
 *   - Maxmin sampling starts at a given node and breaks ties by lowest id.
 *   - If ||x_i - x_q|| = 0 the direction term of the vote is dropped (the vote
 *     is x_q).
 *   - PivotMDS (cited, not defined, in the paper): x = C v for the top two
 *     eigenvectors v of C^T C, C the double-centred squared pivot distances;
 *     each eigenvector's largest-magnitude entry is made positive (entries
 *     within a relative 1e-9 of the largest count as tied; lowest index wins).
 *   - Rescale target: sum over edges of the edge length (m for unit lengths).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_INVAL 1
#define ORC_RANGE 2
#define ORC_DISCONNECTED 3
#define ORC_NOMEM 4

/* ------------------------------------------------------------------ input */

static int cmp_int(const void* a, const void* b) {
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

/* The input is a simple undirected graph (Section 1): symmetric adjacency,
 * no self-loops, no duplicate edges; the method needs it connected (the paper
 * keeps the largest component, Section 4 "Data").  Returns ORC_OK,
 * ORC_INVAL or ORC_DISCONNECTED. */
int orc_validate(int n, const int* rp, const int* ci) {
    if (n < 1 || rp[0] != 0) return ORC_INVAL;
    for (int i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return ORC_INVAL;
    int nnz = rp[n];
    for (int e = 0; e < nnz; ++e)
        if (ci[e] < 0 || ci[e] >= n) return ORC_INVAL;
    int* sorted = (int*)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    if (!sorted) return ORC_NOMEM;
    memcpy(sorted, ci, sizeof(int) * (size_t)nnz);
    for (int i = 0; i < n; ++i)
        qsort(sorted + rp[i], (size_t)(rp[i + 1] - rp[i]), sizeof(int), cmp_int);
    int status = ORC_OK;
    for (int i = 0; i < n && status == ORC_OK; ++i) {
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = sorted[e];
            if (j == i) { status = ORC_INVAL; break; }                  /* loop */
            if (e > rp[i] && sorted[e - 1] == j) { status = ORC_INVAL; break; } /* dup */
            if (!bsearch(&i, sorted + rp[j], (size_t)(rp[j + 1] - rp[j]), sizeof(int), cmp_int)) {
                status = ORC_INVAL; break;                               /* asymmetric */
            }
        }
    }
    free(sorted);
    return status;
}

/* Breadth-first search with a FIFO queue: dist[v] = hop distance from src,
 * -1 if unreached.  Returns the number of reached nodes. */
int orc_bfs(int n, const int* rp, const int* ci, int src, int* dist) {
    int* queue = (int*)malloc(sizeof(int) * (size_t)n);
    for (int v = 0; v < n; ++v) dist[v] = -1;
    int head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int u = queue[head++];
        for (int e = rp[u]; e < rp[u + 1]; ++e) {
            int v = ci[e];
            if (dist[v] < 0) {
                dist[v] = dist[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return tail;
}

/* --------------------------------------------------- pivots and distances */

/* Max/min shortest-path sampling (Section 4.1, "max/min sp"): the first pivot
 * is `first`; the next is the node whose distance to the nearest pivot so far
 * is largest (lowest id on ties).  dist is k x n, row t = BFS from pivots[t].
 * Returns ORC_DISCONNECTED if a BFS misses a node. */
int orc_select_pivots(int n, const int* rp, const int* ci, int k, int first,
                      int* pivots, int* dist) {
    if (k < 1 || k > n || first < 0 || first >= n) return ORC_INVAL;
    int* mind = (int*)malloc(sizeof(int) * (size_t)n);
    for (int v = 0; v < n; ++v) mind[v] = INT32_MAX;
    pivots[0] = first;
    for (int t = 0; t < k; ++t) {
        int* row = dist + (size_t)t * n;
        if (orc_bfs(n, rp, ci, pivots[t], row) != n) { free(mind); return ORC_DISCONNECTED; }
        for (int v = 0; v < n; ++v)
            if (row[v] < mind[v]) mind[v] = row[v];
        if (t + 1 < k) {
            int best = 0;
            for (int v = 1; v < n; ++v)
                if (mind[v] > mind[best]) best = v;
            pivots[t + 1] = best;
        }
    }
    free(mind);
    return ORC_OK;
}

/* dist (k x n) for a given pivot list: one BFS per pivot. */
int orc_bfs_pivots(int n, const int* rp, const int* ci, int k, const int* pivots, int* dist) {
    for (int t = 0; t < k; ++t)
        if (orc_bfs(n, rp, ci, pivots[t], dist + (size_t)t * n) != n) return ORC_DISCONNECTED;
    return ORC_OK;
}

/* ---------------------------------------------------------------- regions */

/* Regions R(p) (Section 3): every node joins the region of its nearest pivot;
 * ties favour the currently smallest region.  Level by level over the
 * nearest-pivot distance l = 0, 1, ...: nodes with a single nearest pivot
 * join it; then every tied node at level l joins the candidate with the
 * smallest (size snapshot taken after the single-candidate joins, rank).
 * Outputs: delta[i] = min_t dist[t][i]; region[i] = pivot rank; size[t];
 * *delta_max = max_i delta[i]. */
int orc_regions(int n, int k, const int* dist, int* delta, int* region, int* size,
                int* delta_max) {
    int* ncand = (int*)malloc(sizeof(int) * (size_t)n);
    int dm = 0;
    for (int i = 0; i < n; ++i) {
        int best = INT32_MAX, cnt = 0;
        for (int t = 0; t < k; ++t) {
            int d = dist[(size_t)t * n + i];
            if (d < best) { best = d; cnt = 1; }
            else if (d == best) cnt++;
        }
        delta[i] = best;
        ncand[i] = cnt;
        region[i] = -1;
        if (best > dm) dm = best;
    }
    /* bucket nodes by delta (stable, ascending id inside a bucket) */
    int* start = (int*)calloc((size_t)dm + 2, sizeof(int));
    int* order = (int*)malloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) start[delta[i] + 1]++;
    for (int l = 0; l <= dm; ++l) start[l + 1] += start[l];
    int* fill = (int*)malloc(sizeof(int) * ((size_t)dm + 1));
    for (int l = 0; l <= dm; ++l) fill[l] = start[l];
    for (int i = 0; i < n; ++i) order[fill[delta[i]]++] = i;
    for (int t = 0; t < k; ++t) size[t] = 0;
    int* snap = (int*)malloc(sizeof(int) * (size_t)k);
    for (int l = 0; l <= dm; ++l) {
        for (int q = start[l]; q < start[l + 1]; ++q) {
            int i = order[q];
            if (ncand[i] != 1) continue;
            for (int t = 0; t < k; ++t)
                if (dist[(size_t)t * n + i] == l) { region[i] = t; size[t]++; break; }
        }
        memcpy(snap, size, sizeof(int) * (size_t)k);
        for (int q = start[l]; q < start[l + 1]; ++q) {
            int i = order[q];
            if (ncand[i] == 1) continue;
            int pick = -1;
            for (int t = 0; t < k; ++t) {
                if (dist[(size_t)t * n + i] != l) continue;
                if (pick < 0 || snap[t] < snap[pick]) pick = t;   /* ascending t: ties keep lower rank */
            }
            region[i] = pick;
        }
        for (int q = start[l]; q < start[l + 1]; ++q) {
            int i = order[q];
            if (ncand[i] != 1) size[region[i]]++;
        }
    }
    *delta_max = dm;
    free(ncand); free(start); free(order); free(fill); free(snap);
    return ORC_OK;
}

/* --------------------------------------------------------- adapted weights */

/* H[t][l] = |{ j in R(p_t) : delta_j <= l }| for l = 0..delta_max (k rows of
 * delta_max+1).  For j in R(p_t), d_{j p_t} = delta_j, so the count s of
 * Section 3 for a node at distance d from p_t is H[t][min(floor(d/2), delta_max)]. */
void orc_histogram(int n, int k, const int* delta, const int* region, int delta_max, int* H) {
    int w = delta_max + 1;
    memset(H, 0, sizeof(int) * (size_t)k * (size_t)w);
    for (int i = 0; i < n; ++i) H[(size_t)region[i] * w + delta[i]]++;
    for (int t = 0; t < k; ++t)
        for (int l = 1; l < w; ++l) H[(size_t)t * w + l] += H[(size_t)t * w + l - 1];
}

/* Adapted weight table (Section 3): w'_ip = s / d_ip^2 with
 * s = |{ j in R(p) : d_jp <= d_ip / 2 }|; zero where no pivot term exists
 * (d < 2).  wtab is k rows of dmax+1 entries indexed by d. */
void orc_weight_table(int k, int delta_max, const int* H, int dmax, double* wtab) {
    int w = delta_max + 1;
    for (int t = 0; t < k; ++t) {
        for (int d = 0; d <= dmax; ++d) {
            double val = 0.0;
            if (d >= 2) {
                int half = d / 2;
                if (half > delta_max) half = delta_max;
                int s = H[(size_t)t * w + half];
                val = (double)s / (double)((int64_t)d * (int64_t)d);
            }
            wtab[(size_t)t * (dmax + 1) + d] = val;
        }
    }
}

/* Denominator of Eq. 5: sum over neighbours of w_ij (= 1 for unit lengths,
 * d_ij = 1), then the pivot weights in ascending pivot rank. */
void orc_denominator(int n, const int* rp, int k, const int* dist, const double* wtab,
                     int dmax, double* den) {
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) s += 1.0;
        for (int t = 0; t < k; ++t) {
            int d = dist[(size_t)t * n + i];
            if (d >= 2) s += wtab[(size_t)t * (dmax + 1) + d];
        }
        den[i] = s;
    }
}

/* ----------------------------------------------------------------- PivotMDS */

/* Double centring of the squared pivot distances:
 * C[i][t] = -1/2 (d_ti^2 - mu_t - nu_i + gamma), mu_t the mean over nodes,
 * nu_i the mean over pivots, gamma the mean of all entries.  C is n x k. */
void orc_pmds_center(int n, int k, const int* dist, double* C) {
    double* mu = (double*)calloc((size_t)k, sizeof(double));
    double gamma = 0.0;
    for (int t = 0; t < k; ++t) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) {
            double d = (double)dist[(size_t)t * n + i];
            s += d * d;
        }
        mu[t] = s / (double)n;
        gamma += s;
    }
    gamma /= (double)n * (double)k;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int t = 0; t < k; ++t) {
            double d = (double)dist[(size_t)t * n + i];
            s += d * d;
        }
        double nu = s / (double)k;
        for (int t = 0; t < k; ++t) {
            double d = (double)dist[(size_t)t * n + i];
            C[(size_t)i * k + t] = -0.5 * (d * d - mu[t] - nu + gamma);
        }
    }
    free(mu);
}

/* M = C^T C, summed over nodes in ascending order. */
void orc_gram(int n, int k, const double* C, double* M) {
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += C[(size_t)i * k + a] * C[(size_t)i * k + b];
            M[(size_t)a * k + b] = s;
        }
}

/* Cyclic Jacobi eigenvalue method for a symmetric k x k matrix (textbook
 * rotations, Rutishauser's formulas).  evals[k]; evecs is k x k with column c
 * the eigenvector of evals[c]; results unsorted.  Returns sweeps used. */
int orc_sym_eig(int k, const double* M, double* evals, double* evecs) {
    double* A = (double*)malloc(sizeof(double) * (size_t)k * k);
    memcpy(A, M, sizeof(double) * (size_t)k * k);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) evecs[(size_t)a * k + b] = (a == b) ? 1.0 : 0.0;
    double fro = 0.0;
    for (size_t q = 0; q < (size_t)k * k; ++q) fro += A[q] * A[q];
    fro = sqrt(fro);
    int sweep;
    for (sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b) off += A[(size_t)a * k + b] * A[(size_t)a * k + b];
        if (sqrt(off) <= 1e-15 * fro || off == 0.0) break;
        for (int p = 0; p < k; ++p) {
            for (int q = p + 1; q < k; ++q) {
                double apq = A[(size_t)p * k + q];
                if (apq == 0.0) continue;
                double app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
                double theta = (aqq - app) / (2.0 * apq);
                double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
                for (int r = 0; r < k; ++r) {         /* A <- A J (columns p, q) */
                    double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
                    A[(size_t)r * k + p] = c * arp - s * arq;
                    A[(size_t)r * k + q] = s * arp + c * arq;
                }
                for (int r = 0; r < k; ++r) {         /* A <- J^T A (rows p, q) */
                    double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
                    A[(size_t)p * k + r] = c * apr - s * aqr;
                    A[(size_t)q * k + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < k; ++r) {         /* V <- V J */
                    double vrp = evecs[(size_t)r * k + p], vrq = evecs[(size_t)r * k + q];
                    evecs[(size_t)r * k + p] = c * vrp - s * vrq;
                    evecs[(size_t)r * k + q] = s * vrp + c * vrq;
                }
            }
        }
    }
    for (int a = 0; a < k; ++a) evals[a] = A[(size_t)a * k + a];
    free(A);
    return sweep;
}

/* PivotMDS: x_i = (C V)_i for V the eigenvectors of C^T C of the two largest
 * eigenvalues (descending); each column's largest-|.| entry is made positive
 * (lowest index among entries within a relative 1e-9 of the largest).  x is n x 2 interleaved; V (k x 2) and lambda (2)
 * are returned as well.  Needs k >= 3 (centring makes C 1 = 0, so rank <= k-1). */
int orc_pivotmds(int n, int k, const int* dist, double* x, double* V, double* lambda) {
    if (k < 3) return ORC_INVAL;
    double* C = (double*)malloc(sizeof(double) * (size_t)n * k);
    double* M = (double*)malloc(sizeof(double) * (size_t)k * k);
    double* ev = (double*)malloc(sizeof(double) * (size_t)k);
    double* E = (double*)malloc(sizeof(double) * (size_t)k * k);
    if (!C || !M || !ev || !E) { free(C); free(M); free(ev); free(E); return ORC_NOMEM; }
    orc_pmds_center(n, k, dist, C);
    orc_gram(n, k, C, M);
    orc_sym_eig(k, M, ev, E);
    int c0 = -1, c1 = -1;
    for (int c = 0; c < k; ++c)
        if (c0 < 0 || ev[c] > ev[c0]) c0 = c;
    for (int c = 0; c < k; ++c)
        if (c != c0 && (c1 < 0 || ev[c] > ev[c1])) c1 = c;
    int cols[2] = {c0, c1};
    for (int a = 0; a < 2; ++a) {
        /* sign rule: the entry of largest magnitude is made positive; entries
         * within a relative 1e-9 of the largest count as tied (ties that are
         * exact in exact arithmetic, as on symmetric graphs, are not exact
         * after rounding) and the lowest index among them decides */
        double mx = 0.0;
        for (int t = 0; t < k; ++t)
            if (fabs(E[(size_t)t * k + cols[a]]) > mx) mx = fabs(E[(size_t)t * k + cols[a]]);
        int big = 0;
        while (big < k - 1 && fabs(E[(size_t)big * k + cols[a]]) < mx * (1.0 - 1e-9)) ++big;
        double sgn = E[(size_t)big * k + cols[a]] < 0.0 ? -1.0 : 1.0;
        for (int t = 0; t < k; ++t) V[t * 2 + a] = sgn * E[(size_t)t * k + cols[a]];
        lambda[a] = ev[cols[a]];
    }
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 2; ++a) {
            double s = 0.0;
            for (int t = 0; t < k; ++t) s += C[(size_t)i * k + t] * V[t * 2 + a];
            x[(size_t)i * 2 + a] = s;
        }
    free(C); free(M); free(ev); free(E);
    return ORC_OK;
}

/* Algorithm 1, rescale step: x <- c x with
 * c = (sum over edges of the edge length) / (sum over edges of ||x_i - x_j||);
 * edges i < j in CSR order, unit lengths. */
int orc_rescale(int n, const int* rp, const int* ci, double* x) {
    double target = 0.0, have = 0.0;
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (j <= i) continue;
            double dx = x[2 * (size_t)i] - x[2 * (size_t)j];
            double dy = x[2 * (size_t)i + 1] - x[2 * (size_t)j + 1];
            target += 1.0;
            have += sqrt(dx * dx + dy * dy);
        }
    if (have == 0.0) return ORC_INVAL;
    double c = target / have;
    for (size_t q = 0; q < 2 * (size_t)n; ++q) x[q] *= c;
    return ORC_OK;
}

/* ------------------------------------------------------------ majorization */

/* One node's Eq. 5 update read from the layout `src`.  Neighbour terms first
 * (w = 1, d = 1): those at a positive distance in CSR order, then those at
 * distance zero; then pivot terms for d >= 2 in ascending rank.
 * vote(q, d) = x_q + d (x_i - x_q) / ||x_i - x_q||, or x_q when the distance
 * is zero.  The paper leaves the order of the sums open.  Putting the
 * zero-distance votes (each equal to x_i) last makes the update of two
 * adjacent nodes with the same position and the same closed neighbourhood
 * identical, as it is in exact arithmetic; summed in CSR order the two would
 * drift apart by rounding alone. */
static void update_node(int i, int n, const int* rp, const int* ci, int k, const int* pivots,
                        const int* dist, const double* wtab, int dmax, const double* den,
                        const double* src, double* out) {
    double xi = src[2 * (size_t)i], yi = src[2 * (size_t)i + 1];
    double nx = 0.0, ny = 0.0;
    int zero = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int j = ci[e];
        double xj = src[2 * (size_t)j], yj = src[2 * (size_t)j + 1];
        double dx = xi - xj, dy = yi - yj;
        double r = sqrt(dx * dx + dy * dy);
        if (r > 0.0) { nx += xj + 1.0 * dx / r; ny += yj + 1.0 * dy / r; }
        else ++zero;
    }
    for (int z = 0; z < zero; ++z) { nx += xi; ny += yi; }
    for (int t = 0; t < k; ++t) {
        int d = dist[(size_t)t * n + i];
        if (d < 2) continue;
        double w = wtab[(size_t)t * (dmax + 1) + d];
        int p = pivots[t];
        double xp = src[2 * (size_t)p], yp = src[2 * (size_t)p + 1];
        double dx = xi - xp, dy = yi - yp;
        double r = sqrt(dx * dx + dy * dy);
        double vx = xp, vy = yp;
        if (r > 0.0) { vx = xp + (double)d * dx / r; vy = yp + (double)d * dy / r; }
        nx += w * vx;
        ny += w * vy;
    }
    out[0] = nx / den[i];
    out[1] = ny / den[i];
}

/* Relative positional change of one sweep x -> y (the test of Algorithm 1's
 * loop).  The stress of Eq. 1 and Eq. 3 and the update of Eq. 5 do not
 * change under a rotation or translation of the whole layout, and with k < n
 * the asymmetric adapted weights leave a steady rigid motion of the layout
 * from sweep to sweep; the change is therefore measured after the best
 * proper rigid motion:
 *   min over rotations R, vectors t of ||y - (R x + t)||_F / ||x - xbar||_F.
 * First pass: the centroids xbar, ybar.  Second pass: with a = x_i - xbar,
 * b = y_i - ybar, P = sum (a.x b.x + a.y b.y), Q = sum (a.x b.y - a.y b.x)
 * and the spread sum |a|^2; the best rotation has cos = P / rho,
 * sin = Q / rho with rho = sqrt(P^2 + Q^2) (no rotation when rho = 0).
 * Third pass: the residual sum |b - R a|^2.  Returns +infinity when the old
 * layout has zero spread (every node at one point). */
double orc_rigid_change(int n, const double* x, const double* y) {
    double sx = 0.0, sy = 0.0, tx = 0.0, ty = 0.0;
    for (int i = 0; i < n; ++i) {
        sx += x[2 * (size_t)i];
        sy += x[2 * (size_t)i + 1];
        tx += y[2 * (size_t)i];
        ty += y[2 * (size_t)i + 1];
    }
    const double mx = sx / n, my = sy / n, nx = tx / n, ny = ty / n;
    double P = 0.0, Q = 0.0, aa = 0.0;
    for (int i = 0; i < n; ++i) {
        const double ax = x[2 * (size_t)i] - mx, ay = x[2 * (size_t)i + 1] - my;
        const double bx = y[2 * (size_t)i] - nx, by = y[2 * (size_t)i + 1] - ny;
        P += ax * bx + ay * by;
        Q += ax * by - ay * bx;
        aa += ax * ax + ay * ay;
    }
    if (!(aa > 0.0)) return INFINITY;
    const double rho = sqrt(P * P + Q * Q);
    const double c = rho > 0.0 ? P / rho : 1.0, s = rho > 0.0 ? Q / rho : 0.0;
    double res = 0.0;
    for (int i = 0; i < n; ++i) {
        const double ax = x[2 * (size_t)i] - mx, ay = x[2 * (size_t)i + 1] - my;
        const double bx = y[2 * (size_t)i] - nx, by = y[2 * (size_t)i + 1] - ny;
        const double ex = bx - (c * ax - s * ay), ey = by - (s * ax + c * ay);
        res += ex * ex + ey * ey;
    }
    return sqrt(res / aa);
}

/* Algorithm 1's loop with the update of Eq. 5.  Jacobi order (every node
 * reads the previous iterate) unless gauss_seidel != 0, which updates in
 * place in ascending node order as Algorithm 1 is written.  Runs `iters`
 * sweeps, or stops after the first sweep whose relative positional change
 * (orc_rigid_change) is at most tol (tol > 0); *iters_done is the number of
 * sweeps run.  Jacobi sweeps may run on `threads` OpenMP threads; the result
 * does not depend on the thread count. */
int orc_majorize(int n, const int* rp, const int* ci, int k, const int* pivots, const int* dist,
                 const double* wtab, int dmax, const double* den, double* x, int iters,
                 double tol, int gauss_seidel, int threads, int* iters_done) {
    double* nxt = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!nxt) return ORC_NOMEM;
    int it;
    for (it = 0; it < iters; ++it) {
        if (gauss_seidel) {
            memcpy(nxt, x, sizeof(double) * 2 * (size_t)n);
            for (int i = 0; i < n; ++i) {
                double o[2];
                update_node(i, n, rp, ci, k, pivots, dist, wtab, dmax, den, x, o);
                x[2 * (size_t)i] = o[0];
                x[2 * (size_t)i + 1] = o[1];
            }
        } else {
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
            for (int i = 0; i < n; ++i)
                update_node(i, n, rp, ci, k, pivots, dist, wtab, dmax, den, x, nxt + 2 * (size_t)i);
        }
        /* the change from the previous iterate (nxt after Gauss-Seidel, x
         * after Jacobi) to the new one */
        const double change = tol > 0.0 ? (gauss_seidel ? orc_rigid_change(n, nxt, x)
                                                        : orc_rigid_change(n, x, nxt))
                                        : INFINITY;
        if (!gauss_seidel) memcpy(x, nxt, sizeof(double) * 2 * (size_t)n);
        if (change <= tol) { ++it; break; }
    }
    free(nxt);
    if (iters_done) *iters_done = it;
    return ORC_OK;
}

/* -------------------------------------------------------------------- stress */

/* Sparse stress s'(x) of Eq. 3: edges i < j in CSR order with w = 1, d = 1,
 * then pivot terms (node ascending, rank ascending, d >= 2) with w'_ip.
 * parts[0] = edge part, parts[1] = pivot part; returns their sum. */
double orc_stress_sparse(int n, const int* rp, const int* ci, int k, const int* pivots,
                         const int* dist, const double* wtab, int dmax, const double* x,
                         double* parts) {
    double se = 0.0, sp = 0.0;
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (j <= i) continue;
            double dx = x[2 * (size_t)i] - x[2 * (size_t)j];
            double dy = x[2 * (size_t)i + 1] - x[2 * (size_t)j + 1];
            double r = sqrt(dx * dx + dy * dy);
            se += (r - 1.0) * (r - 1.0);
        }
    for (int i = 0; i < n; ++i)
        for (int t = 0; t < k; ++t) {
            int d = dist[(size_t)t * n + i];
            if (d < 2) continue;
            int p = pivots[t];
            double dx = x[2 * (size_t)i] - x[2 * (size_t)p];
            double dy = x[2 * (size_t)i + 1] - x[2 * (size_t)p + 1];
            double r = sqrt(dx * dx + dy * dy);
            sp += wtab[(size_t)t * (dmax + 1) + d] * (r - (double)d) * (r - (double)d);
        }
    if (parts) { parts[0] = se; parts[1] = sp; }
    return se + sp;
}

/* Full stress of Eq. 1 with d_ij the hop distance and w_ij = d_ij^-2, pairs
 * i < j, row by row; one BFS per node.  For small graphs only. */
double orc_stress_full(int n, const int* rp, const int* ci, const double* x) {
    int* d = (int*)malloc(sizeof(int) * (size_t)n);
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        orc_bfs(n, rp, ci, i, d);
        for (int j = i + 1; j < n; ++j) {
            double dij = (double)d[j];
            double dx = x[2 * (size_t)i] - x[2 * (size_t)j];
            double dy = x[2 * (size_t)i + 1] - x[2 * (size_t)j + 1];
            double r = sqrt(dx * dx + dy * dy);
            s += (r - dij) * (r - dij) / (dij * dij);
        }
    }
    free(d);
    return s;
}

/* ------------------------------------------------------------ k-means sp
 *
 * Section 4.1, "k-means sp": k pivots are first sampled by max/min sp, then
 * refined by k-means over the shortest-path entries of those pivots.  The
 * paper gives no more detail; the reading implemented here (listed in the
 * design notes):
 *   - node i's feature vector is y_i = (D[0][i], ..., D[k-1][i]), its hop
 *     distances to the k max/min pivots;
 *   - cluster t starts as the single vector y_{p_t} of max/min pivot t;
 *   - Lloyd iterations, at most max_iters (the paper caps its k-means at 50):
 *     every node joins the cluster of the nearest centroid, then every
 *     non-empty cluster's centroid becomes the mean of its members (an empty
 *     cluster keeps its centroid); it stops early when no node changes;
 *   - new pivot t is the node nearest to centroid t, nodes already taken by
 *     a lower t excluded; ties go to the lowest index everywhere.
 * Decisions are made on exact integers wherever the definition allows: a
 * cluster is kept as the integer sum S_t of its members and their count
 * N_t (centroid S_t / N_t); B_ti = y_i . S_t is an exact integer.
 *   - assignment: argmin over t of f_t(i) = a_t - (2 B_ti) / N_t, with
 *     a_t = sum_j (S_tj / N_t)^2 summed over j in ascending order in double
 *     and (2 B_ti) / N_t one correctly rounded double division (||y_i||^2
 *     is common to all t and dropped);
 *   - nearest node to centroid t: argmin over i of N_t ||y_i||^2 - 2 B_ti,
 *     exactly in 64-bit integers.
 * Returns the number of assignment passes run in *iters. */
static double km_a(int k, const int64_t* S, int64_t N) {
    double a = 0.0;
    for (int j = 0; j < k; ++j) {
        double c = (double)S[j] / (double)N;
        a += c * c;
    }
    return a;
}

static int64_t km_dot(int n, int k, const int* D, int i, const int64_t* S) {
    int64_t b = 0;
    for (int j = 0; j < k; ++j) b += (int64_t)D[(size_t)j * n + i] * S[j];
    return b;
}

int orc_kmeans_sp(int n, int k, const int* D, const int* pivots, int max_iters, int* new_pivots,
                  int* assign, int* iters) {
    int64_t* S = (int64_t*)calloc((size_t)k * k, sizeof(int64_t));
    int64_t* S2 = (int64_t*)calloc((size_t)k * k, sizeof(int64_t));
    int64_t* N = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    int64_t* N2 = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    double* a = (double*)malloc(sizeof(double) * (size_t)k);
    char* taken = (char*)calloc((size_t)n, 1);
    if (!S || !S2 || !N || !N2 || !a || !taken) {
        free(S); free(S2); free(N); free(N2); free(a); free(taken);
        return -1;
    }
    for (int t = 0; t < k; ++t) {
        for (int j = 0; j < k; ++j) S[(size_t)t * k + j] = D[(size_t)j * n + pivots[t]];
        N[t] = 1;
    }
    for (int i = 0; i < n; ++i) assign[i] = -1;
    int it = 0;
    while (it < max_iters) {
        ++it;
        for (int t = 0; t < k; ++t) a[t] = km_a(k, S + (size_t)t * k, N[t]);
        int changed = 0;
        for (int i = 0; i < n; ++i) {
            int best = 0;
            double fbest = 0.0;
            for (int t = 0; t < k; ++t) {
                int64_t b = km_dot(n, k, D, i, S + (size_t)t * k);
                double f = a[t] - (2.0 * (double)b) / (double)N[t];
                if (t == 0 || f < fbest) {
                    best = t;
                    fbest = f;
                }
            }
            if (assign[i] != best) ++changed;
            assign[i] = best;
        }
        /* new centroids: member sums; an empty cluster keeps its centroid */
        memset(S2, 0, sizeof(int64_t) * (size_t)k * k);
        memset(N2, 0, sizeof(int64_t) * (size_t)k);
        for (int i = 0; i < n; ++i) {
            int t = assign[i];
            for (int j = 0; j < k; ++j) S2[(size_t)t * k + j] += D[(size_t)j * n + i];
            ++N2[t];
        }
        for (int t = 0; t < k; ++t)
            if (N2[t] > 0) {
                memcpy(S + (size_t)t * k, S2 + (size_t)t * k, sizeof(int64_t) * (size_t)k);
                N[t] = N2[t];
            }
        if (!changed) break;
    }
    /* nearest node to each centroid, in rank order, each node used once */
    for (int t = 0; t < k; ++t) {
        int best = -1;
        int64_t sbest = 0;
        for (int i = 0; i < n; ++i) {
            if (taken[i]) continue;
            int64_t q = 0;
            for (int j = 0; j < k; ++j) {
                int64_t y = D[(size_t)j * n + i];
                q += y * y;
            }
            int64_t sc = N[t] * q - 2 * km_dot(n, k, D, i, S + (size_t)t * k);
            if (best < 0 || sc < sbest) {
                best = i;
                sbest = sc;
            }
        }
        new_pivots[t] = best;
        taken[best] = 1;
    }
    *iters = it;
    free(S); free(S2); free(N); free(N2); free(a); free(taken);
    return 0;
}

/* ------------------------------------------------------------ weighted graphs
 *
 * Algorithm 1's general input: every edge has a positive length (len[e] per
 * arc, equal in both directions).  d_ij is the shortest-path length; the sum
 * along a path is taken from the source outwards in FP64, so d is the least
 * solution of d(s) = 0, d(v) = min over neighbours u of (d(u) + len(u, v))
 * evaluated in floating point.  Edge terms carry w_ij = len^-2 (Eq. 1's
 * weights with d_ij the edge length); pivot terms are as in Section 3 with
 * real distances: w'_ip = s / d_ip^2, s = |{ j in R(p) : d_jp <= d_ip / 2 }|,
 * for every pivot p that is neither i nor a neighbour of i. */

typedef struct { double key; int node; } heap_item;

static void heap_push(heap_item* h, int* size, double key, int node) {
    int c = (*size)++;
    h[c].key = key;
    h[c].node = node;
    while (c > 0) {
        int p = (c - 1) / 2;
        if (h[p].key <= h[c].key) break;
        heap_item t = h[p]; h[p] = h[c]; h[c] = t;
        c = p;
    }
}

static heap_item heap_pop(heap_item* h, int* size) {
    heap_item top = h[0];
    h[0] = h[--(*size)];
    int c = 0;
    for (;;) {
        int l = 2 * c + 1, r = l + 1, m = c;
        if (l < *size && h[l].key < h[m].key) m = l;
        if (r < *size && h[r].key < h[m].key) m = r;
        if (m == c) break;
        heap_item t = h[m]; h[m] = h[c]; h[c] = t;
        c = m;
    }
    return top;
}

/* Dijkstra's algorithm with a binary heap (entries left behind by a later
 * improvement are skipped when popped).  Unreached nodes keep +inf. */
int orc_sssp(int n, const int* rp, const int* ci, const double* len, int src, double* dist) {
    heap_item* h = (heap_item*)malloc(sizeof(heap_item) * ((size_t)rp[n] + 1));
    char* done = (char*)calloc((size_t)n, 1);
    if (!h || !done) { free(h); free(done); return ORC_NOMEM; }
    for (int i = 0; i < n; ++i) dist[i] = INFINITY;
    int size = 0;
    dist[src] = 0.0;
    heap_push(h, &size, 0.0, src);
    while (size > 0) {
        heap_item it = heap_pop(h, &size);
        int u = it.node;
        if (done[u] || it.key != dist[u]) continue;
        done[u] = 1;
        for (int e = rp[u]; e < rp[u + 1]; ++e) {
            int v = ci[e];
            double nd = dist[u] + len[e];
            if (nd < dist[v]) {
                dist[v] = nd;
                heap_push(h, &size, nd, v);
            }
        }
    }
    free(h);
    free(done);
    return ORC_OK;
}

/* max/min sp on weighted distances (Section 4.1): pivots[0] = first; each
 * next pivot is the node with the largest distance to the pivots chosen so
 * far, lowest id on ties.  dist receives the k rows.  ORC_DISCONNECTED when
 * a node is unreachable. */
int orc_select_pivots_w(int n, const int* rp, const int* ci, const double* len, int k, int first,
                        int* pivots, double* dist) {
    double* m = (double*)malloc(sizeof(double) * (size_t)n);
    if (!m) return ORC_NOMEM;
    for (int i = 0; i < n; ++i) m[i] = INFINITY;
    int p = first;
    for (int t = 0; t < k; ++t) {
        pivots[t] = p;
        double* row = dist + (size_t)t * n;
        int st = orc_sssp(n, rp, ci, len, p, row);
        if (st != ORC_OK) { free(m); return st; }
        for (int i = 0; i < n; ++i) {
            if (row[i] == INFINITY) { free(m); return ORC_DISCONNECTED; }
            if (row[i] < m[i]) m[i] = row[i];
        }
        int best = 0;
        for (int i = 1; i < n; ++i)
            if (m[i] > m[best]) best = i;
        p = best;
    }
    free(m);
    return ORC_OK;
}

static const double* g_delta_sort;
static int cmp_delta_id(const void* a, const void* b) {
    int i = *(const int*)a, j = *(const int*)b;
    double di = g_delta_sort[i], dj = g_delta_sort[j];
    if (di < dj) return -1;
    if (di > dj) return 1;
    return (i > j) - (i < j);
}

/* Regions by rule R1 on real distances: delta_i = min_t dist[t][i]; the
 * candidates of i are the ranks at exactly that distance.  Levels are the
 * distinct delta values in ascending order; in a level the single-candidate
 * nodes join first, then each tied node joins the candidate with the
 * smallest (size snapshot, rank). */
int orc_regions_w(int n, int k, const double* dist, double* delta, int* region, int* size) {
    int* ncand = (int*)malloc(sizeof(int) * (size_t)n);
    int* order = (int*)malloc(sizeof(int) * (size_t)n);
    int* snap = (int*)malloc(sizeof(int) * (size_t)k);
    if (!ncand || !order || !snap) { free(ncand); free(order); free(snap); return ORC_NOMEM; }
    for (int i = 0; i < n; ++i) {
        double best = INFINITY;
        int cnt = 0;
        for (int t = 0; t < k; ++t) {
            double d = dist[(size_t)t * n + i];
            if (d < best) { best = d; cnt = 1; }
            else if (d == best) cnt++;
        }
        delta[i] = best;
        ncand[i] = cnt;
        region[i] = -1;
        order[i] = i;
    }
    g_delta_sort = delta;
    qsort(order, (size_t)n, sizeof(int), cmp_delta_id);
    for (int t = 0; t < k; ++t) size[t] = 0;
    for (int a = 0; a < n;) {
        int b = a;
        while (b < n && delta[order[b]] == delta[order[a]]) ++b;   /* level [a, b) */
        double l = delta[order[a]];
        for (int q = a; q < b; ++q) {
            int i = order[q];
            if (ncand[i] != 1) continue;
            for (int t = 0; t < k; ++t)
                if (dist[(size_t)t * n + i] == l) { region[i] = t; size[t]++; break; }
        }
        memcpy(snap, size, sizeof(int) * (size_t)k);
        for (int q = a; q < b; ++q) {
            int i = order[q];
            if (ncand[i] == 1) continue;
            int pick = -1;
            for (int t = 0; t < k; ++t) {
                if (dist[(size_t)t * n + i] != l) continue;
                if (pick < 0 || snap[t] < snap[pick]) pick = t;
            }
            region[i] = pick;
        }
        for (int q = a; q < b; ++q) {
            int i = order[q];
            if (ncand[i] != 1) size[region[i]]++;
        }
        a = b;
    }
    free(ncand); free(order); free(snap);
    return ORC_OK;
}

/* Pivot-term weights w[t][i] (0 where no term exists: p_t = i or p_t a
 * neighbour of i) and denominators den_i = sum over i's arcs in CSR order of
 * len^-2, then sum over ranks ascending of w[t][i].  s counts the members j of
 * R(p_t) with delta_j <= d / 2 by scanning the region's member list. */
int orc_terms_w(int n, const int* rp, const int* ci, const double* len, int k, const int* pivots,
                const double* dist, const double* delta, const int* region, double* w, double* den) {
    int* start = (int*)calloc((size_t)k + 1, sizeof(int));
    int* members = (int*)malloc(sizeof(int) * (size_t)n);
    int* fill = (int*)malloc(sizeof(int) * ((size_t)k + 1));
    if (!start || !members || !fill) { free(start); free(members); free(fill); return ORC_NOMEM; }
    for (int i = 0; i < n; ++i) start[region[i] + 1]++;
    for (int t = 0; t < k; ++t) start[t + 1] += start[t];
    for (int t = 0; t <= k; ++t) fill[t] = start[t];
    for (int i = 0; i < n; ++i) members[fill[region[i]]++] = i;
    for (int t = 0; t < k; ++t) {
        int p = pivots[t];
        for (int i = 0; i < n; ++i) {
            double val = 0.0;
            int adjacent = 0;
            for (int e = rp[i]; e < rp[i + 1]; ++e) adjacent |= ci[e] == p;
            if (i != p && !adjacent) {
                double d = dist[(size_t)t * n + i];
                int s = 0;
                for (int q = start[t]; q < start[t + 1]; ++q) s += delta[members[q]] <= d / 2.0;
                val = (double)s / (d * d);
            }
            w[(size_t)t * n + i] = val;
        }
    }
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) s += 1.0 / (len[e] * len[e]);
        for (int t = 0; t < k; ++t) s += w[(size_t)t * n + i];
        den[i] = s;
    }
    free(start); free(members); free(fill);
    return ORC_OK;
}

/* Eq. 5 with lengths, one node from `src`: neighbour votes at a positive
 * distance in CSR order, w_e (x_j + len (x_i - x_j) / r) with w_e = len^-2;
 * then the zero-distance neighbour votes w_e x_i in CSR order; then pivot
 * terms by ascending rank, w (x_p + d (x_i - x_p) / r), or w x_p at r = 0. */
static void update_node_w(int i, const int* rp, const int* ci, const double* len, int n, int k,
                          const int* pivots, const double* dist, const double* w, const double* den,
                          const double* src, double* out) {
    double xi = src[2 * (size_t)i], yi = src[2 * (size_t)i + 1];
    double nx = 0.0, ny = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int j = ci[e];
        double dx = xi - src[2 * (size_t)j], dy = yi - src[2 * (size_t)j + 1];
        double r = sqrt(dx * dx + dy * dy);
        if (r > 0.0) {
            double we = 1.0 / (len[e] * len[e]);
            nx += we * (src[2 * (size_t)j] + (len[e] * dx) / r);
            ny += we * (src[2 * (size_t)j + 1] + (len[e] * dy) / r);
        }
    }
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int j = ci[e];
        double dx = xi - src[2 * (size_t)j], dy = yi - src[2 * (size_t)j + 1];
        double r = sqrt(dx * dx + dy * dy);
        if (!(r > 0.0)) {
            double we = 1.0 / (len[e] * len[e]);
            nx += we * xi;
            ny += we * yi;
        }
    }
    for (int t = 0; t < k; ++t) {
        double wt = w[(size_t)t * n + i];
        if (wt == 0.0) continue;
        int p = pivots[t];
        double d = dist[(size_t)t * n + i];
        double px = src[2 * (size_t)p], py = src[2 * (size_t)p + 1];
        double dx = xi - px, dy = yi - py;
        double r = sqrt(dx * dx + dy * dy);
        double vx = px, vy = py;
        if (r > 0.0) {
            vx = px + d * dx / r;
            vy = py + d * dy / r;
        }
        nx += wt * vx;
        ny += wt * vy;
    }
    out[2 * (size_t)i] = nx / den[i];
    out[2 * (size_t)i + 1] = ny / den[i];
}

/* `iters` Jacobi sweeps of Eq. 5 with lengths, in place on x (n x 2). */
int orc_majorize_w(int n, const int* rp, const int* ci, const double* len, int k, const int* pivots,
                   const double* dist, const double* w, const double* den, double* x, int iters) {
    double* y = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!y) return ORC_NOMEM;
    for (int it = 0; it < iters; ++it) {
        for (int i = 0; i < n; ++i) update_node_w(i, rp, ci, len, n, k, pivots, dist, w, den, x, y);
        memcpy(x, y, sizeof(double) * 2 * (size_t)n);
    }
    free(y);
    return ORC_OK;
}

/* s'(x) of Eq. 3 with lengths: edges (i < j) len^-2 (r - len)^2, then every
 * pivot term w (r - d)^2, in node order. */
double orc_stress_w(int n, const int* rp, const int* ci, const double* len, int k, const int* pivots,
                    const double* dist, const double* w, const double* x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (j <= i) continue;
            double dx = x[2 * (size_t)i] - x[2 * (size_t)j], dy = x[2 * (size_t)i + 1] - x[2 * (size_t)j + 1];
            double r = sqrt(dx * dx + dy * dy);
            s += (r - len[e]) * (r - len[e]) / (len[e] * len[e]);
        }
        for (int t = 0; t < k; ++t) {
            double wt = w[(size_t)t * n + i];
            if (wt == 0.0) continue;
            int p = pivots[t];
            double dx = x[2 * (size_t)i] - x[2 * (size_t)p], dy = x[2 * (size_t)i + 1] - x[2 * (size_t)p + 1];
            double r = sqrt(dx * dx + dy * dy);
            double d = dist[(size_t)t * n + i];
            s += wt * (r - d) * (r - d);
        }
    }
    return s;
}

/* PivotMDS on real distances: C_it = -1/2 (d^2 - mu_t - nu_i + gamma) as for
 * hop distances; the rest as orc_pivotmds. */
int orc_pivotmds_w(int n, int k, const double* dist, double* x, double* V, double* lambda) {
    if (k < 3) return ORC_INVAL;
    double* C = (double*)malloc(sizeof(double) * (size_t)n * k);
    double* mu = (double*)calloc((size_t)k, sizeof(double));
    double* M = (double*)malloc(sizeof(double) * (size_t)k * k);
    double* ev = (double*)malloc(sizeof(double) * (size_t)k);
    double* E = (double*)malloc(sizeof(double) * (size_t)k * k);
    if (!C || !mu || !M || !ev || !E) { free(C); free(mu); free(M); free(ev); free(E); return ORC_NOMEM; }
    double gamma = 0.0;
    for (int t = 0; t < k; ++t) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) { double d = dist[(size_t)t * n + i]; s += d * d; }
        mu[t] = s / (double)n;
        gamma += s;
    }
    gamma /= (double)n * (double)k;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int t = 0; t < k; ++t) { double d = dist[(size_t)t * n + i]; s += d * d; }
        double nu = s / (double)k;
        for (int t = 0; t < k; ++t) {
            double d = dist[(size_t)t * n + i];
            C[(size_t)i * k + t] = -0.5 * (d * d - mu[t] - nu + gamma);
        }
    }
    orc_gram(n, k, C, M);
    orc_sym_eig(k, M, ev, E);
    int c0 = -1, c1 = -1;
    for (int c = 0; c < k; ++c)
        if (c0 < 0 || ev[c] > ev[c0]) c0 = c;
    for (int c = 0; c < k; ++c)
        if (c != c0 && (c1 < 0 || ev[c] > ev[c1])) c1 = c;
    int cols[2] = {c0, c1};
    for (int a = 0; a < 2; ++a) {
        double mx = 0.0;
        for (int t = 0; t < k; ++t)
            if (fabs(E[(size_t)t * k + cols[a]]) > mx) mx = fabs(E[(size_t)t * k + cols[a]]);
        int big = 0;
        while (big < k - 1 && fabs(E[(size_t)big * k + cols[a]]) < mx * (1.0 - 1e-9)) ++big;
        double sgn = E[(size_t)big * k + cols[a]] < 0.0 ? -1.0 : 1.0;
        for (int t = 0; t < k; ++t) V[t * 2 + a] = sgn * E[(size_t)t * k + cols[a]];
        lambda[a] = ev[cols[a]];
    }
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 2; ++a) {
            double s = 0.0;
            for (int t = 0; t < k; ++t) s += C[(size_t)i * k + t] * V[t * 2 + a];
            x[(size_t)i * 2 + a] = s;
        }
    free(C); free(mu); free(M); free(ev); free(E);
    return ORC_OK;
}

/* Rescale with lengths: c = (sum of edge lengths) / (sum of drawn edge
 * lengths), edges i < j in CSR order. */
int orc_rescale_w(int n, const int* rp, const int* ci, const double* len, double* x) {
    double target = 0.0, have = 0.0;
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (j <= i) continue;
            double dx = x[2 * (size_t)i] - x[2 * (size_t)j];
            double dy = x[2 * (size_t)i + 1] - x[2 * (size_t)j + 1];
            target += len[e];
            have += sqrt(dx * dx + dy * dy);
        }
    if (have == 0.0) return ORC_INVAL;
    double c = target / have;
    for (size_t q = 0; q < 2 * (size_t)n; ++q) x[q] *= c;
    return ORC_OK;
}
