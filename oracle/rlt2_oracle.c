/*
 * Plain FP64 CPU oracle of the level-2 RLT dual ascent for the QAP
 * (arXiv 1510.02065).  TEST INFRASTRUCTURE ONLY: used by the tests, the
 * smoke check and the benchmark's CPU-baseline leg; never by the GPU library.
 *
 * The code is written for being checked by eye against the paper, not for
 * speed: dense index arithmetic, no blocking, no fusion.  Parallel loops only
 * split work whose pieces touch disjoint data, so the results do not depend
 * on the thread count.  Compile without FMA contraction (-ffp-contract=off).
 */
#include "rlt2_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops that follow (results do not depend on it). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ========================================================================== */
/* Linear assignment problem (Section 4.1: cost concentration is a LAP).       */
/* ========================================================================== */

/*
 * Successive shortest augmenting paths (the Hungarian method in its
 * shortest-path form).  Row potentials u and column potentials v keep every
 * reduced cost M[r][c] - u[r] - v[c] non-negative and the matched ones zero.
 * Each free row f is inserted by a Dijkstra search over columns on reduced
 * costs; when the search reaches an unmatched column the potentials of the
 * scanned part of the tree are shifted and the path is flipped.
 */
double oracle_lap_solve(int n, const double* M, int* row2col)
{
    if (n <= 0) return 0.0;
    double* u = (double*)calloc((size_t)n, sizeof(double));
    double* v = (double*)calloc((size_t)n, sizeof(double));
    double* dist = (double*)malloc((size_t)n * sizeof(double));
    int* col2row = (int*)malloc((size_t)n * sizeof(int));
    int* pred = (int*)malloc((size_t)n * sizeof(int));
    char* done = (char*)malloc((size_t)n);

    for (int r = 0; r < n; ++r) row2col[r] = -1;
    for (int c = 0; c < n; ++c) col2row[c] = -1;

    for (int f = 0; f < n; ++f) {
        for (int c = 0; c < n; ++c) {
            dist[c] = M[(size_t)f * n + c] - u[f] - v[c];
            pred[c] = f;
            done[c] = 0;
        }
        int sink = -1;
        double dsink = 0.0;
        while (sink < 0) {
            int c = -1;
            for (int cc = 0; cc < n; ++cc)
                if (!done[cc] && (c < 0 || dist[cc] < dist[c])) c = cc;
            done[c] = 1;
            if (col2row[c] < 0) {
                sink = c;
                dsink = dist[c];
                break;
            }
            int r = col2row[c];
            for (int cc = 0; cc < n; ++cc) {
                if (done[cc]) continue;
                double nd = dist[c] + (M[(size_t)r * n + cc] - u[r] - v[cc]);
                if (nd < dist[cc]) {
                    dist[cc] = nd;
                    pred[cc] = r;
                }
            }
        }
        /* Shift potentials of the scanned tree so matched reduced costs stay 0
         * and every reduced cost stays >= 0. */
        u[f] += dsink;
        for (int c = 0; c < n; ++c) {
            if (!done[c] || c == sink) continue;
            double shift = dsink - dist[c];
            v[c] -= shift;
            u[col2row[c]] += shift;
        }
        /* Flip the augmenting path ending at the sink. */
        int c = sink;
        for (;;) {
            int r = pred[c];
            int next = row2col[r];
            row2col[r] = c;
            col2row[c] = r;
            if (r == f) break;
            c = next;
        }
    }

    double total = 0.0;
    for (int r = 0; r < n; ++r) total += M[(size_t)r * n + row2col[r]];
    free(u); free(v); free(dist); free(col2row); free(pred); free(done);
    return total;
}

/*
 * Canonical dual of the optimal dual face.  Complementary slackness with an
 * optimal assignment sigma gives
 *   column form: v_q - v_c <= M[s][q] - M[s][c]   with s = sigma^-1(c),
 *   row form:    u_r - u_s <= M[r][c] - M[s][c]   with c = sigma(s),
 * and both systems are independent of which optimal sigma is used.  The
 * greatest solution with all values <= 0 is the vector of shortest-path
 * distances from a virtual source joined to every node by a zero-weight arc;
 * Bellman-Ford with n-1 rounds computes it.  The other half of each dual
 * point is the row (column) minimum of M minus that vector.
 */
void oracle_lap_canonical_dual(int n, const double* M, const int* row2col,
                               double* uc, double* vc, double* ur, double* vr)
{
    int* col2row = (int*)malloc((size_t)n * sizeof(int));
    for (int r = 0; r < n; ++r) col2row[row2col[r]] = r;

    /* column-canonical point */
    for (int q = 0; q < n; ++q) vc[q] = 0.0;
    for (int round = 0; round + 1 < n; ++round) {
        for (int c = 0; c < n; ++c) {
            int s = col2row[c];
            for (int q = 0; q < n; ++q) {
                double w = M[(size_t)s * n + q] - M[(size_t)s * n + c];
                double cand = vc[c] + w;
                if (cand < vc[q]) vc[q] = cand;
            }
        }
    }
    for (int r = 0; r < n; ++r) {
        double m = M[(size_t)r * n] - vc[0];
        for (int q = 1; q < n; ++q) {
            double t = M[(size_t)r * n + q] - vc[q];
            if (t < m) m = t;
        }
        uc[r] = m;
    }

    /* row-canonical point */
    for (int r = 0; r < n; ++r) ur[r] = 0.0;
    for (int round = 0; round + 1 < n; ++round) {
        for (int s = 0; s < n; ++s) {
            int c = row2col[s];
            for (int r = 0; r < n; ++r) {
                double w = M[(size_t)r * n + c] - M[(size_t)s * n + c];
                double cand = ur[s] + w;
                if (cand < ur[r]) ur[r] = cand;
            }
        }
    }
    for (int q = 0; q < n; ++q) {
        double m = M[q] - ur[0];
        for (int r = 1; r < n; ++r) {
            double t = M[(size_t)r * n + q] - ur[r];
            if (t < m) m = t;
        }
        vr[q] = m;
    }
    free(col2row);
}

/*
 * Concentrate one block (Section 4.1): S is moved to the parent coefficient
 * and every entry is replaced by its residual.  The residual is the mean of
 * the residuals under the two canonical dual points; each of those is >= 0
 * exactly because the subtracted dual is a row (column) minimum of the
 * already-rounded differences.
 */
double oracle_lap_concentrate(int n, const double* M, double* R,
                              double* duals, int* row2col_out)
{
    if (n <= 0) return 0.0;
    int* row2col = (int*)malloc((size_t)n * sizeof(int));
    double* buf = (double*)malloc((size_t)4 * n * sizeof(double));
    double *uc = buf, *vc = buf + n, *ur = buf + 2 * n, *vr = buf + 3 * n;

    oracle_lap_solve(n, M, row2col);
    oracle_lap_canonical_dual(n, M, row2col, uc, vc, ur, vr);

    double s_uc = 0.0, s_vc = 0.0, s_ur = 0.0, s_vr = 0.0;
    for (int r = 0; r < n; ++r) s_uc += uc[r];
    for (int q = 0; q < n; ++q) s_vc += vc[q];
    for (int r = 0; r < n; ++r) s_ur += ur[r];
    for (int q = 0; q < n; ++q) s_vr += vr[q];
    double S = 0.5 * ((s_uc + s_vc) + (s_ur + s_vr));

    for (int r = 0; r < n; ++r) {
        for (int q = 0; q < n; ++q) {
            double m = M[(size_t)r * n + q];
            double r1 = (m - vc[q]) - uc[r];
            double r2 = (m - ur[r]) - vr[q];
            R[(size_t)r * n + q] = 0.5 * (r1 + r2);
        }
    }
    if (duals) memcpy(duals, buf, (size_t)4 * n * sizeof(double));
    if (row2col_out) memcpy(row2col_out, row2col, (size_t)n * sizeof(int));
    free(row2col);
    free(buf);
    return S;
}

/* ========================================================================== */
/* RLT2 dual ascent (Section 4, Algorithm 1).                                  */
/* ========================================================================== */

struct oracle_rlt2 {
    int N;
    double LB, lbprime;
    double* B;   /* [i][j]                 */
    double* C;   /* [i][j][k][n]           */
    double* D;   /* [i][j][k][n][p][q]     */
    double* SD;  /* value moved D_ijkn -> c_ijkn by the last step 4 */
    double* SC;  /* value moved C_ij -> b_ij by the last step 6 / iteration 0 */
};

#define IDX2(N, i, j) ((size_t)(i) * (N) + (j))
#define IDX4(N, i, j, k, n) ((((size_t)(i) * (N) + (j)) * (N) + (k)) * (N) + (n))
#define IDX6(N, i, j, k, n, p, q) \
    ((((IDX4(N, i, j, k, n)) * (N) + (p)) * (N)) + (q))

int oracle_rlt2_N(const oracle_rlt2* s) { return s->N; }
double oracle_rlt2_lb(const oracle_rlt2* s) { return s->LB; }
double oracle_rlt2_last_lbprime(const oracle_rlt2* s) { return s->lbprime; }
double* oracle_rlt2_B(oracle_rlt2* s) { return s->B; }
double* oracle_rlt2_C(oracle_rlt2* s) { return s->C; }
double* oracle_rlt2_D(oracle_rlt2* s) { return s->D; }
double* oracle_rlt2_SD(oracle_rlt2* s) { return s->SD; }
double* oracle_rlt2_SC(oracle_rlt2* s) { return s->SC; }
void oracle_rlt2_set_lb(oracle_rlt2* s, double lb) { s->LB = lb; }

void oracle_rlt2_free(oracle_rlt2* s)
{
    if (!s) return;
    free(s->B); free(s->C); free(s->D); free(s->SD); free(s->SC);
    free(s);
}

/* Initialisation lines of Algorithm 1 (before the loop). */
oracle_rlt2* oracle_rlt2_new(int N, const double* F, const double* Dm,
                             const double* B0, double constant)
{
    if (N < 3 || !F || !Dm) return NULL;
    oracle_rlt2* s = (oracle_rlt2*)calloc(1, sizeof(*s));
    if (!s) return NULL;
    size_t n2 = (size_t)N * N, n4 = n2 * n2, n6 = n4 * n2;
    s->N = N;
    s->B = (double*)calloc(n2, sizeof(double));
    s->C = (double*)calloc(n4, sizeof(double));
    s->D = (double*)calloc(n6, sizeof(double));
    s->SD = (double*)calloc(n4, sizeof(double));
    s->SC = (double*)calloc(n2, sizeof(double));
    if (!s->B || !s->C || !s->D || !s->SD || !s->SC) {
        oracle_rlt2_free(s);
        return NULL;
    }
    s->LB = constant;
    s->lbprime = 0.0;
    /* b_ij: cost of placing facility i at location j (the diagonal flow times
     * the diagonal distance, plus any linear cost given by the caller). */
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double b = F[IDX2(N, i, i)] * Dm[IDX2(N, j, j)];
            if (B0) b = b + B0[IDX2(N, i, j)];
            s->B[IDX2(N, i, j)] = b;
        }
    /* c_ijkn = f_ik * d_jn, i != k, j != n. */
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            for (int k = 0; k < N; ++k) {
                if (k == i) continue;
                for (int n = 0; n < N; ++n) {
                    if (n == j) continue;
                    s->C[IDX4(N, i, j, k, n)] = F[IDX2(N, i, k)] * Dm[IDX2(N, j, n)];
                }
            }
    /* d = 0 (calloc). */
    return s;
}

/* Concentrate C_ij -> b_ij for every (i, j): rows k != i, columns n != j,
 * both in ascending original index. */
static void concentrate_C_to_B(oracle_rlt2* s)
{
    const int N = s->N, m = N - 1;
#pragma omp parallel
    {
        double* M = (double*)malloc((size_t)m * m * sizeof(double));
        double* R = (double*)malloc((size_t)m * m * sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int ij = 0; ij < N * N; ++ij) {
            int i = ij / N, j = ij % N;
            int r = 0;
            for (int k = 0; k < N; ++k) {
                if (k == i) continue;
                int c = 0;
                for (int n = 0; n < N; ++n) {
                    if (n == j) continue;
                    M[(size_t)r * m + c] = s->C[IDX4(N, i, j, k, n)];
                    ++c;
                }
                ++r;
            }
            double S = oracle_lap_concentrate(m, M, R, NULL, NULL);
            r = 0;
            for (int k = 0; k < N; ++k) {
                if (k == i) continue;
                int c = 0;
                for (int n = 0; n < N; ++n) {
                    if (n == j) continue;
                    s->C[IDX4(N, i, j, k, n)] = R[(size_t)r * m + c];
                    ++c;
                }
                ++r;
            }
            s->SC[IDX2(N, i, j)] = S;
            s->B[IDX2(N, i, j)] += S;
        }
        free(M);
        free(R);
    }
}

/* Concentrate B -> LB' (the N x N assignment over the whole of B). */
static double concentrate_B(oracle_rlt2* s)
{
    const int N = s->N;
    double* R = (double*)malloc((size_t)N * N * sizeof(double));
    double S = oracle_lap_concentrate(N, s->B, R, NULL, NULL);
    memcpy(s->B, R, (size_t)N * N * sizeof(double));
    free(R);
    return S;
}

void oracle_rlt2_iteration0(oracle_rlt2* s)
{
    concentrate_C_to_B(s);
    s->lbprime = concentrate_B(s);
    s->LB += s->lbprime;
}

/* Step 1 -- cost spreading B -> C (Section 4.2): each c_ijkn, k != i,
 * n != j, receives b_ij / (N-1); then b = 0. */
static void spread_B_to_C(oracle_rlt2* s)
{
    const int N = s->N;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double share = s->B[IDX2(N, i, j)] / (double)(N - 1);
            for (int k = 0; k < N; ++k) {
                if (k == i) continue;
                for (int n = 0; n < N; ++n) {
                    if (n == j) continue;
                    s->C[IDX4(N, i, j, k, n)] += share;
                }
            }
            s->B[IDX2(N, i, j)] = 0.0;
        }
}

/* Step 2 -- cost spreading C -> D (Section 4.2): each d_ijknpq, p not in
 * {i,k}, q not in {j,n}, receives c_ijkn / (N-2); then c = 0. */
static void spread_C_to_D(oracle_rlt2* s)
{
    const int N = s->N;
#pragma omp parallel for schedule(static)
    for (int ij = 0; ij < N * N; ++ij) {
        int i = ij / N, j = ij % N;
        for (int k = 0; k < N; ++k) {
            if (k == i) continue;
            for (int n = 0; n < N; ++n) {
                if (n == j) continue;
                double share = s->C[IDX4(N, i, j, k, n)] / (double)(N - 2);
                for (int p = 0; p < N; ++p) {
                    if (p == i || p == k) continue;
                    for (int q = 0; q < N; ++q) {
                        if (q == j || q == n) continue;
                        s->D[IDX6(N, i, j, k, n, p, q)] += share;
                    }
                }
                s->C[IDX4(N, i, j, k, n)] = 0.0;
            }
        }
    }
}

/* Step 3 -- transfer between the six complementary coefficients of D
 * (constraint family of equation (11), operation of Section 4.3).  The paper
 * fixes only that the transfer is zero-sum; the equal split is used: each of
 * the six members becomes their mean.  The three (facility, location) pairs
 * are ordered by facility index, P1 < P2 < P3, and the six members are summed
 * in lexicographic order of the permutation of (P1, P2, P3). */
static void transfer_D(oracle_rlt2* s)
{
    const int N = s->N;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < N; ++i) {
        for (int k = i + 1; k < N; ++k)
            for (int p = k + 1; p < N; ++p)
                for (int j = 0; j < N; ++j)
                    for (int n = 0; n < N; ++n) {
                        if (n == j) continue;
                        for (int q = 0; q < N; ++q) {
                            if (q == j || q == n) continue;
                            /* pairs P1=(i,j) P2=(k,n) P3=(p,q) */
                            size_t m0 = IDX6(N, i, j, k, n, p, q); /* P1 P2 P3 */
                            size_t m1 = IDX6(N, i, j, p, q, k, n); /* P1 P3 P2 */
                            size_t m2 = IDX6(N, k, n, i, j, p, q); /* P2 P1 P3 */
                            size_t m3 = IDX6(N, k, n, p, q, i, j); /* P2 P3 P1 */
                            size_t m4 = IDX6(N, p, q, i, j, k, n); /* P3 P1 P2 */
                            size_t m5 = IDX6(N, p, q, k, n, i, j); /* P3 P2 P1 */
                            double sum = s->D[m0];
                            sum += s->D[m1];
                            sum += s->D[m2];
                            sum += s->D[m3];
                            sum += s->D[m4];
                            sum += s->D[m5];
                            double mean = sum / 6.0;
                            s->D[m0] = mean; s->D[m1] = mean; s->D[m2] = mean;
                            s->D[m3] = mean; s->D[m4] = mean; s->D[m5] = mean;
                        }
                    }
    }
}

/* Step 4 -- cost concentration D -> C (Section 4.1): block D_ijkn has rows
 * p not in {i,k} and columns q not in {j,n}, in ascending original index;
 * c_ijkn += S and the block is replaced by its residuals. */
static void concentrate_D_to_C(oracle_rlt2* s)
{
    const int N = s->N, m = N - 2;
#pragma omp parallel
    {
        double* M = (double*)malloc((size_t)m * m * sizeof(double));
        double* R = (double*)malloc((size_t)m * m * sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int ij = 0; ij < N * N; ++ij) {
            int i = ij / N, j = ij % N;
            for (int k = 0; k < N; ++k) {
                if (k == i) continue;
                for (int n = 0; n < N; ++n) {
                    if (n == j) continue;
                    int r = 0;
                    for (int p = 0; p < N; ++p) {
                        if (p == i || p == k) continue;
                        int c = 0;
                        for (int q = 0; q < N; ++q) {
                            if (q == j || q == n) continue;
                            M[(size_t)r * m + c] = s->D[IDX6(N, i, j, k, n, p, q)];
                            ++c;
                        }
                        ++r;
                    }
                    double S = oracle_lap_concentrate(m, M, R, NULL, NULL);
                    r = 0;
                    for (int p = 0; p < N; ++p) {
                        if (p == i || p == k) continue;
                        int c = 0;
                        for (int q = 0; q < N; ++q) {
                            if (q == j || q == n) continue;
                            s->D[IDX6(N, i, j, k, n, p, q)] = R[(size_t)r * m + c];
                            ++c;
                        }
                        ++r;
                    }
                    s->SD[IDX4(N, i, j, k, n)] = S;
                    s->C[IDX4(N, i, j, k, n)] += S;
                }
            }
        }
        free(M);
        free(R);
    }
}

/* Step 5 -- transfer between the two complementary coefficients of C
 * (equation (10), Section 4.3), equal split: c_ijkn = c_knij = their mean. */
static void transfer_C(oracle_rlt2* s)
{
    const int N = s->N;
    for (int i = 0; i < N; ++i)
        for (int k = i + 1; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int n = 0; n < N; ++n) {
                    if (n == j) continue;
                    size_t a = IDX4(N, i, j, k, n), b = IDX4(N, k, n, i, j);
                    double mean = (s->C[a] + s->C[b]) / 2.0;
                    s->C[a] = mean;
                    s->C[b] = mean;
                }
}

void oracle_rlt2_step(oracle_rlt2* s, int step)
{
    switch (step) {
    case 1: spread_B_to_C(s); break;
    case 2: spread_C_to_D(s); break;
    case 3: transfer_D(s); break;
    case 4: concentrate_D_to_C(s); break;
    case 5: transfer_C(s); break;
    case 6: concentrate_C_to_B(s); break;
    case 7: s->lbprime = concentrate_B(s); break;
    case 8: s->LB += s->lbprime; break;
    default: break;
    }
}

void oracle_rlt2_iterate(oracle_rlt2* s, int T)
{
    for (int t = 0; t < T; ++t)
        for (int step = 1; step <= 8; ++step) oracle_rlt2_step(s, step);
}
