/*
 * Plain FP64 CPU oracle for the level-2 RLT dual ascent on the Quadratic
 * Assignment Problem (Goncalves, Pessoa, Drummond, Bentes, Farias,
 * arXiv 1510.02065).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the
 * smoke check and the CPU-baseline leg of the benchmark have an obviously
 * correct reference to compare the GPU library against.  It shares no code,
 * header, table or helper with the GPU path, and the GPU path never calls it.
 *
 * Storage is deliberately naive: B is N x N, C is a dense N^4 array indexed
 * [i][j][k][n] and D a dense N^6 array indexed [i][j][k][n][p][q]; entries
 * whose facility or location indices repeat are never read or written.
 *
 * Every per-step function follows one line of Algorithm 1 of the paper; the
 * cost concentration follows Section 4.1, spreading Section 4.2, and the
 * transfer between complementary coefficients Section 4.3 (under the equal
 * split reading documented in the source).
 */
#ifndef RLT2_ORACLE_H
#define RLT2_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- linear assignment (Section 4.1) -------------------------------------- */

/* Optimal assignment of an n x n row-major matrix by successive shortest
 * augmenting paths.  row2col[r] receives the column of row r.  Returns
 * sum_r M[r][row2col[r]]. */
double oracle_lap_solve(int n, const double* M, int* row2col);

/* Canonical optimal dual of M given an optimal assignment row2col, by two
 * Bellman-Ford runs on the difference-constraint graphs of the optimal dual
 * face.  Writes the column-canonical point (uc, vc) and the row-canonical
 * point (ur, vr); each array has n entries. */
void oracle_lap_canonical_dual(int n, const double* M, const int* row2col,
                               double* uc, double* vc, double* ur, double* vr);

/* Cost concentration of one block: R <- residual of M under the averaged
 * canonical dual, returns the transferred value S.  duals (nullable) receives
 * [uc | vc | ur | vr] (4n values), row2col (nullable) the assignment used. */
double oracle_lap_concentrate(int n, const double* M, double* R,
                              double* duals, int* row2col);

/* ---- RLT2 dual ascent (Section 4, Algorithm 1) ---------------------------- */

typedef struct oracle_rlt2 oracle_rlt2;

/* Initial dual state: LB = constant, b_ij = f_ii d_jj (+ B0_ij),
 * c_ijkn = f_ik d_jn, d = 0.  B0 may be NULL.  Returns NULL on bad input or
 * allocation failure. */
oracle_rlt2* oracle_rlt2_new(int N, const double* F, const double* D,
                             const double* B0, double constant);
void oracle_rlt2_free(oracle_rlt2* s);

/* Iteration 0: concentrate every C_ij into b_ij, then B into LB. */
void oracle_rlt2_iteration0(oracle_rlt2* s);

/* One numbered step of the Algorithm 1 loop body (1..8). */
void oracle_rlt2_step(oracle_rlt2* s, int step);

/* T full loop iterations (steps 1..8 each). */
void oracle_rlt2_iterate(oracle_rlt2* s, int T);

int     oracle_rlt2_N(const oracle_rlt2* s);
double  oracle_rlt2_lb(const oracle_rlt2* s);
double  oracle_rlt2_last_lbprime(const oracle_rlt2* s);
/* Direct views of the dense state arrays (B: N^2, C: N^4, D: N^6) and of the
 * transferred values recorded by the last concentrations (SD: N^4 for step 4,
 * SC: N^2 for step 6 or iteration 0). */
double* oracle_rlt2_B(oracle_rlt2* s);
double* oracle_rlt2_C(oracle_rlt2* s);
double* oracle_rlt2_D(oracle_rlt2* s);
double* oracle_rlt2_SD(oracle_rlt2* s);
double* oracle_rlt2_SC(oracle_rlt2* s);
void    oracle_rlt2_set_lb(oracle_rlt2* s, double lb);

/* Number of OpenMP threads the oracle runs with (1 when built without it). */
int oracle_threads(void);
/* Set the OpenMP thread count of the parallel loops (n >= 1). */
void oracle_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
