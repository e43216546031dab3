// Linear assignment with canonical dual on gfx950: the solver of every
// assignment kernel (the concentrations and the batched qap_lap_solve).
//
// Cost concentration (Section 4.1 of arXiv 1510.02065) solves one assignment
// problem per block of the reduced-cost array, moves its value S to the
// parent coefficient and replaces the block by its residuals.  Here a segment
// of SEG lanes owns one n x n problem (n <= SEG*K) whose matrix sits in LDS;
// lane l holds the K columns (and, in the row passes, the K rows)
// l, l+SEG, ..., l+(K-1)*SEG.  A wave carries 64/SEG problems.  Every
// Dijkstra step scans K columns per lane and then needs only a log2(SEG)-level
// argmin, so the fixed per-step cost (argmin, broadcast, bookkeeping) is
// shared by more columns and more problems than with one column per lane.
//
// Solver: the Hungarian method in its shortest-augmenting-path form
// (Munkres), started from the two-sided reduction (u_r = row minimum of M,
// v_c = column minimum of M - u) and a greedy matching on its zero reduced
// costs (see lap_reduce_start).  Each remaining free row is inserted by
// Dijkstra over columns with absolute tentative distances; the duals of the
// scanned tree are shifted once when an unmatched column is reached.  Ties are
// broken towards the lowest column index.
//
// Residual: the optimal dual is not unique, so the residual is taken under a
// canonical choice that does not depend on the solver's path:
//   column point: v^c = the greatest v <= 0 on the optimal dual face,
//                 u^c_r = min_q (M_rq - v^c_q);
//   row point:    u^r = the greatest u <= 0 on the optimal dual face,
//                 v^r_q = min_r (M_rq - u^r_r);
//   R = ((M - v^c - u^c) + (M - u^r - v^r)) / 2,
//   S = (sum u^c + sum v^c + sum u^r + sum v^r) / 2.
// With the solver's duals (u, v) and assignment sigma, v^c - v is the vector
// of shortest distances in the column graph whose arc c -> q costs the reduced
// cost M[sigma^-1(c)][q] - u - v >= 0, starting from label -v_q at every
// column: one dense Dijkstra pass.  The row point is the same on the row graph.
// With round-to-nearest arithmetic (FP64, or FP32 nearest) both residual
// halves are >= 0 exactly, because the subtracted dual is a row (column)
// minimum of the already rounded differences.  The FP32 certified variant is
// described at its code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lap_wave.hpp"
#include "rlt2_kernels.hpp"

namespace qap {

// Segment collectives for SEG in {8, 16, 32, 64} lanes (all lanes of a
// segment active; segments independent).
template <int SEG>
struct SegS {
    static_assert(SEG == 8 || SEG == 16 || SEG == 32 || SEG == 64, "segment size");
    __device__ __forceinline__ static int lane() { return threadIdx.x & (SEG - 1); }

    template <typename T>
    __device__ __forceinline__ static T min(T x) {
        x = tmin(x, dpp<kDppXor1>(x));
        x = tmin(x, dpp<kDppXor2>(x));
        x = tmin(x, dpp<kDppHalfMirror>(x));
        if constexpr (SEG >= 16) x = tmin(x, dpp<kDppMirror>(x));
        if constexpr (SEG >= 32) {
            T a, b;
            swap_pair<16>(x, a, b);
            x = tmin(a, b);
        }
        if constexpr (SEG >= 64) {
            T a, b;
            swap_pair<32>(x, a, b);
            x = tmin(a, b);
        }
        return x;
    }
    __device__ __forceinline__ static int imin(int x) {
        x = ::min(x, dpp_i<kDppXor1>(x));
        x = ::min(x, dpp_i<kDppXor2>(x));
        x = ::min(x, dpp_i<kDppHalfMirror>(x));
        if constexpr (SEG >= 16) x = ::min(x, dpp_i<kDppMirror>(x));
        if constexpr (SEG >= 32) {
            const unsigned u = (unsigned)x;
            auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
            x = ::min((int)r[0], (int)r[1]);
        }
        if constexpr (SEG >= 64) {
            const unsigned u = (unsigned)x;
            auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
            x = ::min((int)r[0], (int)r[1]);
        }
        return x;
    }
};

// Sum of one value per column over the 64 column slots of a problem, in one
// fixed order whatever the layout: column l + k*SEG lives in slot k of lane l;
// pairs at stride 1, 2, 4, ..., 32 are added bottom-up (the segment
// butterflies give every lane the same bits at each level, since addition is
// commutative), absent columns count as +0 and the levels above SEG*K add
// +0 explicitly.  So every (SEG, K) configuration returns the same bits.
template <int SEG, int K, typename T, typename Add>
__device__ __forceinline__ T tree_sum64(const T (&x)[K], Add add)
{
    constexpr int KP = K <= 1 ? 1 : K <= 2 ? 2 : K <= 4 ? 4 : 8;
    static_assert(SEG * KP <= 64, "at most 64 column slots");
    T y[KP];
    for (int s = 0; s < KP; ++s) y[s] = s < K ? x[s] : T(0);
    for (int s = 0; s < KP; ++s) {
        T v = y[s];
        v = add(v, dpp<kDppXor1>(v));
        v = add(v, dpp<kDppXor2>(v));
        v = add(v, dpp<kDppHalfMirror>(v));
        if constexpr (SEG >= 16) v = add(v, dpp<kDppMirror>(v));
        if constexpr (SEG >= 32) {
            T a, b;
            swap_pair<16>(v, a, b);
            v = add(a, b);
        }
        if constexpr (SEG >= 64) {
            T a, b;
            swap_pair<32>(v, a, b);
            v = add(a, b);
        }
        y[s] = v;
    }
    for (int st = 1; st < KP; st *= 2)
        for (int s = 0; s + st < KP; s += 2 * st) y[s] = add(y[s], y[s + st]);
    for (int w = SEG * KP; w < 64; w *= 2) y[0] = add(y[0], T(0));
    return y[0];
}

// Per-problem LDS working set, for a problem of size n:
// [matrix n x n of T, row stride ld = n | 1 | aux: n ints | p: n shorts |
//  way: n shorts | pad | u: n doubles | vb: n doubles].  The odd row stride
// puts the rows a lane-per-row access reads (lane r reading row r) on
// distinct LDS banks; with an even n, lanes whose rows lie a multiple of
// 64 / gcd(n, 64) banks' worth apart would hit the same bank.  The LDS a wave needs bounds how many
// waves a CU holds, and the assignment kernels run faster the more it holds,
// so the arrays hold the n columns only (every write is guarded by c < n),
// row and path indices (< 64 * 64) are 16-bit, and no array is kept that
// another one can stand in for.
template <typename T, int SEG, int K>
struct SlotLds {
    __host__ __device__ static int row_stride(int n) { return n | 1; }
    __host__ __device__ static size_t mat_bytes(int n) {
        return (((size_t)n * row_stride(n) * sizeof(T)) + 15) & ~(size_t)15;
    }
    __host__ __device__ static size_t idx_bytes(int n) {
        return (((size_t)n * sizeof(int) + 2 * (size_t)n * sizeof(short)) + 15) & ~(size_t)15;
    }
    __host__ __device__ static size_t vec_bytes(int n) { return idx_bytes(n) + 2 * (size_t)n * sizeof(double); }
    __host__ __device__ static size_t bytes(int n) { return mat_bytes(n) + vec_bytes(n); }
};

template <typename T, int SEG, int K>
struct SlotScratch {
    T* M;
    int ld;      // row stride of M (odd)
    int* aux;    // row ownership, then sigma (column of row r)
    short* p;    // row matched to column c (or -1); the flat solver keeps r*ld
    short* way;  // predecessor column on the shortest path
    double* u;   // n doubles: the FP64 scratch of the certified completion and the auction
    double* vb;  // n doubles after u, likewise
    // The same two arrays as values of type T, used by every other phase (for
    // FP32, their first halves): ut[c] = dual of the row matched to column c,
    // vt = row minima in the start, then column duals in the canonical passes.
    // A phase reads an array only through the view it was written through.
    T* ut;
    T* vt;
    __device__ SlotScratch(unsigned char* base, int n) {
        const size_t mb = SlotLds<T, SEG, K>::mat_bytes(n);
        M = reinterpret_cast<T*>(base);
        ld = SlotLds<T, SEG, K>::row_stride(n);
        aux = reinterpret_cast<int*>(base + mb);
        p = reinterpret_cast<short*>(aux + n);
        way = p + n;
        u = reinterpret_cast<double*>(base + mb + SlotLds<T, SEG, K>::idx_bytes(n));
        vb = u + n;
        ut = reinterpret_cast<T*>(u);
        vt = reinterpret_cast<T*>(vb);
    }
};

template <typename T, int SEG, int K, bool DOWN>
__device__ __forceinline__ double lap_complete(const SlotScratch<T, SEG, K>& sc, int n, T* __restrict__ R,
                                               long long ldr, T* __restrict__ duals, int32_t* __restrict__ assign,
                                               const T (&vc)[K], const T (&ur)[K], const int (&sg)[K]);

// Canonical dual and residual, from the solver's optimal duals and matching:
// v (column duals) and p (row matched to each column) of this lane's K
// columns, ucol the dual of that row; the LDS copies sc.p (row indices) and
// sc.ut (row dual per column) hold the same for every column.
template <typename T, int SEG, int K, bool DOWN>
__device__ __forceinline__ double lap_canonical_finish(const SlotScratch<T, SEG, K>& sc, int n,
                                                       T* __restrict__ R, long long ldr, T* __restrict__ duals,
                                                       int32_t* __restrict__ assign, const T (&v)[K],
                                                       const int (&p)[K], const T (&ucol)[K])
{
    using S = SegS<SEG>;
    constexpr int NONE = 1 << 20;   // larger than any column index
    const T* __restrict__ M = sc.M;
    const int ldm = sc.ld;   // row stride of M
    const int lane = S::lane();
    const T INF = inf_of<T>();
    int c[K];
    bool ok[K];
    for (int s = 0; s < K; ++s) {
        c[s] = s * SEG + lane;
        ok[s] = c[s] < n;
    }

    // ---- column-canonical point (lanes = columns) ---------------------------
    // x_q = shortest distance to column q from label -v_q at every column, over
    // arcs c -> q of reduced cost M[p(c)][q] - u_{p(c)} - v_q >= 0.
    T x[K];
    {
        bool done[K];
        for (int s = 0; s < K; ++s) {
            x[s] = ok[s] ? -v[s] : INF;
            done[s] = !ok[s];
        }
        for (int step = 0; step < n; ++step) {
            T lm = INF;
            int lc = NONE;
            for (int s = 0; s < K; ++s)
                if (!done[s] && x[s] < lm) {
                    lm = x[s];
                    lc = c[s];
                }
            const T dmin = S::min(lm);
            const int cc = S::imin(lm == dmin ? lc : NONE);
            if (cc >= n) break;
            const int r = sc.p[cc];
            const T ur = sc.ut[cc];
            for (int s = 0; s < K; ++s) {
                done[s] = done[s] || (c[s] == cc);
                const T nd = dmin + ((M[r * ldm + (ok[s] ? c[s] : 0)] - ur) - v[s]);
                if (!done[s] && nd < x[s]) x[s] = nd;
            }
        }
        for (int s = 0; s < K; ++s)
            if (!ok[s]) x[s] = 0;
    }

    // sigma (column of row r) in sc.aux, v in sc.vt; the solver's row dual
    // u_r is the dual stored at column sigma(r).
    wave_sync();
    for (int s = 0; s < K; ++s) {
        if (ok[s] && p[s] >= 0) sc.aux[p[s]] = c[s];
        if (ok[s]) sc.vt[c[s]] = v[s];
    }
    wave_sync();
    int sg[K];     // lane as rows: sigma of this lane's rows
    T urow[K];
    for (int s = 0; s < K; ++s) {
        sg[s] = ok[s] ? sc.aux[c[s]] : 0;
        urow[s] = sc.ut[sg[s]];
    }

    // ---- row-canonical point (lanes = rows) ---------------------------------
    // y_r = shortest distance to row r from label -u_r at every row, over
    // arcs s -> r of reduced cost M[r][sigma(s)] - v_{sigma(s)} - u_r >= 0.
    T y[K];
    {
        bool done[K];
        for (int s = 0; s < K; ++s) {
            y[s] = ok[s] ? -urow[s] : INF;
            done[s] = !ok[s];
        }
        for (int step = 0; step < n; ++step) {
            T lm = INF;
            int lc = NONE;
            for (int s = 0; s < K; ++s)
                if (!done[s] && y[s] < lm) {
                    lm = y[s];
                    lc = c[s];
                }
            const T dmin = S::min(lm);
            const int rr = S::imin(lm == dmin ? lc : NONE);
            if (rr >= n) break;
            const int cs = sc.aux[rr];
            const T vcs = sc.vt[cs];
            for (int s = 0; s < K; ++s) {
                done[s] = done[s] || (c[s] == rr);
                const T nd = dmin + ((M[(ok[s] ? c[s] : 0) * ldm + cs] - vcs) - urow[s]);
                if (!done[s] && nd < y[s]) y[s] = nd;
            }
        }
        for (int s = 0; s < K; ++s)
            if (!ok[s]) y[s] = 0;
    }
    T vc[K], ur[K];
    for (int s = 0; s < K; ++s) {
        vc[s] = v[s] + x[s];     // lane as columns
        ur[s] = urow[s] + y[s];  // lane as rows
    }
    return lap_complete<T, SEG, K, DOWN>(sc, n, R, ldr, duals, assign, vc, ur, sg);
}

// From the canonical points to the residual and S: vc (this lane's columns'
// column-canonical duals), ur (its rows' row-canonical duals) and sg (sigma of
// its rows, for `assign`).  The other halves of the two points are completed
// here: u^c_r = min_q (M_rq - v^c_q), v^r_q = min_r (M_rq - u^r_r).
// DOWN selects the FP32 certified completion (every written value rounded
// toward -inf); otherwise the completion runs in T with round-to-nearest and
// S is summed in FP64.
template <typename T, int SEG, int K, bool DOWN>
__device__ __forceinline__ double lap_complete(const SlotScratch<T, SEG, K>& sc, int n, T* __restrict__ R,
                                               long long ldr, T* __restrict__ duals, int32_t* __restrict__ assign,
                                               const T (&vc)[K], const T (&ur)[K], const int (&sg)[K])
{
    using S = SegS<SEG>;
    const T* __restrict__ M = sc.M;
    const int ldm = sc.ld;   // row stride of M
    const int lane = S::lane();
    const T INF = inf_of<T>();
    int c[K];
    bool ok[K];
    for (int s = 0; s < K; ++s) {
        c[s] = s * SEG + lane;
        ok[s] = c[s] < n;
    }
    wave_sync();

    if constexpr (!DOWN) {
        // ---- round to nearest: residual = mean of the residuals under the
        // two points ----
        for (int s = 0; s < K; ++s) {
            if (!ok[s]) continue;
            sc.ut[c[s]] = vc[s];
            sc.vt[c[s]] = ur[s];
        }
        wave_sync();
        T uc[K], vr[K];   // uc: lane as rows; vr: lane as columns
        for (int s = 0; s < K; ++s) {
            uc[s] = INF;
            vr[s] = INF;
            if (ok[s]) {
                for (int q = 0; q < n; ++q) uc[s] = tmin(uc[s], M[c[s] * ldm + q] - sc.ut[q]);
                for (int r = 0; r < n; ++r) vr[s] = tmin(vr[s], M[r * ldm + c[s]] - sc.vt[r]);
            }
        }
        wave_sync();
        for (int s = 0; s < K; ++s)
            if (ok[s]) sc.ut[c[s]] = uc[s];
        wave_sync();
        if (R != nullptr) {
            for (int s = 0; s < K; ++s) {
                if (!ok[s]) continue;
                T* Rr = R + c[s];
                for (int r = 0; r < n; ++r, Rr += ldr) {
                    const T m = M[r * ldm + c[s]];
                    const T r1 = (m - vc[s]) - sc.ut[r];
                    const T r2 = (m - sc.vt[r]) - vr[s];
                    *Rr = (T)0.5 * (r1 + r2);
                }
            }
        }
        double xuc[K], xvc[K], xur[K], xvr[K];
        for (int s = 0; s < K; ++s) {
            xuc[s] = ok[s] ? (double)uc[s] : 0.0;
            xvc[s] = ok[s] ? (double)vc[s] : 0.0;
            xur[s] = ok[s] ? (double)ur[s] : 0.0;
            xvr[s] = ok[s] ? (double)vr[s] : 0.0;
            if (!ok[s]) continue;
            if (duals != nullptr) {
                duals[c[s]] = uc[s];
                duals[n + c[s]] = vc[s];
                duals[2 * n + c[s]] = ur[s];
                duals[3 * n + c[s]] = vr[s];
            }
            if (assign != nullptr) assign[c[s]] = sg[s];
        }
        auto plus = [](double a, double b) { return a + b; };
        const double suc = tree_sum64<SEG, K>(xuc, plus);
        const double svc = tree_sum64<SEG, K>(xvc, plus);
        const double sur = tree_sum64<SEG, K>(xur, plus);
        const double svr = tree_sum64<SEG, K>(xvr, plus);
        wave_sync();
        return 0.5 * ((suc + svc) + (sur + svr));
    } else {
        // ---- FP32 certified: the duals are completed in FP64 so that they
        // stay feasible (u_r + v_q <= M_rq exactly).  With U = (uc + ur)/2
        // and V = (vc + vr)/2 the residual M - U - V (the same value as the
        // mean of the two residuals) is then >= 0, and each entry and
        // S = sum U + sum V are written rounded down.
        //
        // A completed dual is a minimum of differences t = M - d.  Each
        // difference is computed once in round-to-nearest FP64, within
        // 2^-53 |t| of the exact one; as t - 2^-53 |t| increases with t, the
        // minimum m of the computed differences lowered by 2^-50 |m| (the
        // lowering itself rounding by at most 2^-53 of the result) lies below
        // every exact difference.  A residual entry M - V - U is computed in
        // two round-to-nearest steps, within 2.01 * 2^-53 (|M| + |V| + |U|)
        // of the exact value; lowered by 2^-50 times that sum (the lowering's
        // own rounding included), then by the float conversion toward -inf,
        // and clamped at 0 (the exact residual is >= 0), it is a valid lower
        // value.  Both replace per-operation directed rounding (TwoSum) with
        // a margin far below one FP32 step.
        for (int s = 0; s < K; ++s) {
            if (!ok[s]) continue;
            sc.u[c[s]] = (double)vc[s];
            sc.vb[c[s]] = (double)ur[s];
        }
        wave_sync();
        double uc[K], vr[K], U[K], V[K];
        for (int s = 0; s < K; ++s) {
            uc[s] = __builtin_huge_val();
            vr[s] = __builtin_huge_val();
            if (ok[s]) {
                for (int q = 0; q < n; ++q)
                    uc[s] = __builtin_fmin(uc[s], (double)M[c[s] * ldm + q] - sc.u[q]);
                for (int r = 0; r < n; ++r)
                    vr[s] = __builtin_fmin(vr[s], (double)M[r * ldm + c[s]] - sc.vb[r]);
                uc[s] -= __builtin_fabs(uc[s]) * 0x1p-50;
                vr[s] -= __builtin_fabs(vr[s]) * 0x1p-50;
            }
            U[s] = ok[s] ? 0.5 * add_down(uc[s], (double)ur[s]) : 0.0;   // lane as rows
            V[s] = ok[s] ? 0.5 * add_down((double)vc[s], vr[s]) : 0.0;   // lane as columns
        }
        wave_sync();
        for (int s = 0; s < K; ++s)
            if (ok[s]) sc.u[c[s]] = U[s];
        wave_sync();
        if (R != nullptr) {
            for (int s = 0; s < K; ++s) {
                if (!ok[s]) continue;
                T* Rr = R + c[s];
                const double aV = __builtin_fabs(V[s]) * 0x1p-50;
                for (int r = 0; r < n; ++r, Rr += ldr) {
                    const double m = (double)M[r * ldm + c[s]];
                    const double ur_ = sc.u[r];
                    const double t = (m - V[s]) - ur_;
                    // 2^-50 (|M| + |U| + |V|), the sum rounded once before
                    // the FMA and once in it: >= (1 - 2^-52) of the exact one.
                    const double margin = __builtin_fma(__builtin_fabs(m) + __builtin_fabs(ur_), 0x1p-50, aV);
                    *Rr = to_float_down_nonneg(__builtin_fmax(t - margin, 0.0));
                }
            }
        }
        for (int s = 0; s < K; ++s) {
            if (!ok[s]) continue;
            if (duals != nullptr) {
                duals[c[s]] = (T)uc[s];
                duals[n + c[s]] = vc[s];
                duals[2 * n + c[s]] = ur[s];
                duals[3 * n + c[s]] = (T)vr[s];
            }
            if (assign != nullptr) assign[c[s]] = sg[s];
        }
        // S = sum U + sum V rounded down: each sum over the 64 column slots
        // is taken in round-to-nearest (six levels of pairwise additions, so
        // within (1 + 2^-53)^6 - 1 < 7 * 2^-53 of the exact sum relative to
        // the sum of magnitudes) and lowered by 2^-48 times the
        // round-to-nearest sum of the magnitudes, which covers that error and
        // the lowering's own rounding.
        auto plus = [](double a, double b) { return a + b; };
        double aU[K], aV[K];
        for (int s = 0; s < K; ++s) {
            aU[s] = __builtin_fabs(U[s]);
            aV[s] = __builtin_fabs(V[s]);
        }
        const double su = tree_sum64<SEG, K>(U, plus), sau = tree_sum64<SEG, K>(aU, plus);
        const double sv = tree_sum64<SEG, K>(V, plus), sav = tree_sum64<SEG, K>(aV, plus);
        wave_sync();
        return add_down(su - sau * 0x1p-48, sv - sav * 0x1p-48);
    }
}

// Start of both solvers.  Row minima u_r of M, then column minima v_c of the
// reduced rows M_rc - u_r (the two-sided reduction: every reduced cost is
// >= 0 and each row and column has a zero), then a matching on the zeros:
// the columns in index order each take the lowest still free row r with
// M_rc - u_r = v_c.  On the structured blocks of the dual ascent this leaves
// far fewer rows free than a column reduction alone, and every free row costs
// Dijkstra steps.  Lane layout as in lap_concentrate_slots (c[s] = this
// lane's columns, which are also its rows).  On return sc.vt[r] = u_r for every
// row r < n, kept through the Hungarian phase (a free row enters with that
// dual); v[s] and row[s] (matched row or -1) for each of the lane's columns;
// the result is the mask of matched rows (bit r).  sc.u is used as scratch.
template <typename T, int SEG, int K>
__device__ __forceinline__ unsigned long long lap_reduce_start(const SlotScratch<T, SEG, K>& sc, int n,
                                                               const int (&c)[K], const bool (&ok)[K], T (&v)[K],
                                                               int (&row)[K])
{
    // Each loop reads kReduceChunk LDS entries before it uses any of them, so
    // a lane waits for LDS once per chunk; whole chunks first, whose offsets
    // are the chunk's base plus constants, then the last partial one (indices
    // past n - 1 re-read entry n - 1, which changes no minimum and sets no new
    // bit).  Zero masks are
    // 32-bit when a problem has at most 32 columns.  The minima are fmin (one
    // instruction in FP64 where a select takes three; equal values can differ
    // only in the sign of a zero, which no later comparison or sum sees), the
    // zero masks selects rather than branches, and row offsets are 24-bit
    // products (n <= 64).
    constexpr int kReduceChunk = 8;
    using Mask = std::conditional_t<(SEG * K <= 32), unsigned, unsigned long long>;
    const T* __restrict__ M = sc.M;
    const int ldm = sc.ld;   // row stride of M
    for (int s = 0; s < K; ++s) {
        if (!ok[s]) continue;
        const T* __restrict__ Mr = M + __umul24(c[s], ldm);
        T um = Mr[0];
        int q0 = 0;
        for (; q0 + kReduceChunk <= n; q0 += kReduceChunk) {
            T m[kReduceChunk];
#pragma unroll
            for (int e = 0; e < kReduceChunk; ++e) m[e] = Mr[q0 + e];
#pragma unroll
            for (int e = 0; e < kReduceChunk; ++e) um = tmin(m[e], um);
        }
        if (q0 < n) {
            T m[kReduceChunk];
#pragma unroll
            for (int e = 0; e < kReduceChunk; ++e) m[e] = Mr[min(q0 + e, n - 1)];
#pragma unroll
            for (int e = 0; e < kReduceChunk; ++e) um = tmin(m[e], um);
        }
        sc.vt[c[s]] = um;
    }
    wave_sync();
    Mask zc[K];   // zero mask of each of this lane's columns
    for (int s = 0; s < K; ++s) {
        v[s] = 0;
        row[s] = -1;
        zc[s] = 0;
        if (!ok[s]) continue;
        const T* __restrict__ Mc = M + c[s];
        T vm = Mc[0] - sc.vt[0];
        Mask z = 1;
        int r0 = 0;
        for (; r0 + kReduceChunk <= n; r0 += kReduceChunk) {
            const T* __restrict__ Mc0 = Mc + __umul24(r0, ldm);
            const T* __restrict__ u0 = sc.vt + r0;
            T x[kReduceChunk];
#pragma unroll
            for (int e = 0; e < kReduceChunk; ++e) x[e] = Mc0[e * ldm] - u0[e];
#pragma unroll
            for (int e = 0; e < kReduceChunk; ++e) {
                const Mask bit = Mask(1) << (r0 + e);
                const bool lt = x[e] < vm, eq = x[e] == vm;
                z = lt ? bit : (eq ? (z | bit) : z);
                vm = tmin(x[e], vm);
            }
        }
        if (r0 < n) {
            T x[kReduceChunk];
#pragma unroll
            for (int e = 0; e < kReduceChunk; ++e) {
                const int r = min(r0 + e, n - 1);
                x[e] = Mc[__umul24(r, ldm)] - sc.vt[r];
            }
#pragma unroll
            for (int e = 0; e < kReduceChunk; ++e) {
                const Mask bit = Mask(1) << min(r0 + e, n - 1);
                const bool lt = x[e] < vm, eq = x[e] == vm;
                z = lt ? bit : (eq ? (z | bit) : z);
                vm = tmin(x[e], vm);
            }
        }
        v[s] = vm;
        zc[s] = z;
    }
    if constexpr (K == 1) {
        // One column per lane: the greedy matching runs on the scalar unit,
        // each segment's column q read from its lane q.  The rows taken before
        // column q are written to lane q, which afterwards takes the lowest of
        // its zero rows outside that set (the row the scalar loop gave it).
        constexpr int LPW = 64 / SEG;
        const int seg = (threadIdx.x & 63) / SEG;
        Mask tk[LPW];
        int ns[LPW];
        int nmax = 0;
#pragma unroll
        for (int g = 0; g < LPW; ++g) {
            tk[g] = 0;
            ns[g] = __builtin_amdgcn_readlane(n, g * SEG);
            nmax = ::max(nmax, ns[g]);
        }
        const int wl = threadIdx.x & 63;
        Mask before = 0;   // rows taken before this lane's column
        for (int q = 0; q < nmax; ++q) {
#pragma unroll
            for (int g = 0; g < LPW; ++g) {
                if (q >= ns[g]) continue;
                const int ln = g * SEG + q;
                Mask z;
                if constexpr (sizeof(Mask) == 4) {
                    z = (Mask)__builtin_amdgcn_readlane((int)zc[0], ln);
                } else {
                    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)zc[0], ln);
                    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(zc[0] >> 32), ln);
                    z = ((Mask)hi << 32) | lo;
                }
                before = wl == ln ? tk[g] : before;
                z &= ~tk[g];
                tk[g] |= z & (Mask(0) - z);   // its lowest set bit
            }
        }
        const Mask mine = zc[0] & ~before;
        const int rowv = mine ? (sizeof(Mask) == 4 ? __builtin_ctz((unsigned)mine)
                                                   : __builtin_ctzll((unsigned long long)mine))
                              : -1;
        row[0] = ok[0] ? rowv : -1;
        Mask taken = tk[0];
#pragma unroll
        for (int g = 1; g < LPW; ++g)
            if (seg == g) taken = tk[g];
        wave_sync();
        return (unsigned long long)taken;
    } else {
        Mask* __restrict__ zeros = reinterpret_cast<Mask*>(sc.u);
        for (int s = 0; s < K; ++s)
            if (ok[s]) zeros[c[s]] = zc[s];
        wave_sync();
        Mask taken = 0;
        for (int q0 = 0; q0 < n; q0 += kReduceChunk) {
            Mask zq[kReduceChunk];
#pragma unroll
            for (int e = 0; e < kReduceChunk; ++e) zq[e] = zeros[min(q0 + e, n - 1)];
#pragma unroll
            for (int e = 0; e < kReduceChunk; ++e) {
                const int q = q0 + e;
                if (q >= n) break;
                const Mask z = zq[e] & ~taken;
                const int r = z ? (sizeof(Mask) == 4 ? __builtin_ctz((unsigned)z)
                                                     : __builtin_ctzll((unsigned long long)z))
                                : -1;
                if (r >= 0) taken |= Mask(1) << r;
                for (int s = 0; s < K; ++s)
                    if (c[s] == q) row[s] = r;
            }
        }
        wave_sync();
        return (unsigned long long)taken;
    }
}

// Solve, canonicalise and write residuals for the n x n matrix sc.M (in LDS,
// row stride n, left unchanged).  R (nullable) receives the residual (row
// stride ldr), duals (nullable) [uc | vc | ur | vr], assign (nullable) the
// solver's assignment.
// Returns S to every lane of the segment.  Called by whole waves; segments may
// have different n (0 <= n <= SEG*K).
template <typename T, int SEG, int K, bool DOWN>
__device__ __forceinline__ double lap_concentrate_slots(const SlotScratch<T, SEG, K>& sc, int n,
                                                        T* __restrict__ R, long long ldr, T* __restrict__ duals,
                                                        int32_t* __restrict__ assign)
{
    using S = SegS<SEG>;
    constexpr int NONE = 1 << 20;   // larger than any column index
    const T* __restrict__ M = sc.M;
    const int ldm = sc.ld;   // row stride of M
    const int lane = S::lane();
    const T INF = inf_of<T>();

    int c[K];      // this lane's columns (also its rows in the row passes)
    bool ok[K];
    for (int s = 0; s < K; ++s) {
        c[s] = s * SEG + lane;
        ok[s] = c[s] < n;
    }

    // ---- two-sided reduction and greedy start -------------------------------
    T v[K];        // column duals
    int p[K];      // row matched to each column (or -1)
    T ucol[K];     // dual of that row
    const unsigned long long taken = lap_reduce_start<T, SEG, K>(sc, n, c, ok, v, p);
    for (int s = 0; s < K; ++s) {
        ucol[s] = p[s] >= 0 ? sc.vt[p[s]] : (T)0;
        if (!ok[s]) continue;
        sc.p[c[s]] = p[s];
        sc.ut[c[s]] = ucol[s];
        sc.aux[c[s]] = ((taken >> c[s]) & 1ull) ? 0 : NONE;   // lane as row c[s]
    }
    wave_sync();

    // ---- Hungarian method for the rows left free -----------------------------
    for (int i = 0; i < n; ++i) {
        if (sc.aux[i] != NONE) continue;   // row i already matched
        T dist[K];
        int way[K];
        bool used[K];
        for (int s = 0; s < K; ++s) {
            dist[s] = INF;
            way[s] = -1;
            used[s] = false;
        }
        int i0 = i;     // row being scanned
        const T ufree = sc.vt[i];   // dual of the free row (its row minimum)
        T ui0 = ufree;  // dual of the row being scanned
        T d0 = 0;       // distance at which row i0 was reached
        int j0 = -1;    // column through which row i0 was reached
        int jend = -1;
        T dend = 0;
        for (int pass = 0; pass <= n; ++pass) {
            T lm = INF;
            int lc = NONE;
            for (int s = 0; s < K; ++s) {
                const bool live = ok[s] && !used[s];
                const T cur = d0 + ((M[i0 * ldm + (ok[s] ? c[s] : 0)] - ui0) - v[s]);
                if (live && cur < dist[s]) {
                    dist[s] = cur;
                    way[s] = j0;
                }
                if (live && dist[s] < lm) {
                    lm = dist[s];
                    lc = c[s];
                }
            }
            const T dmin = S::min(lm);
            const int j1 = S::imin(lm == dmin ? lc : NONE);
            const int j1c = j1 < n ? j1 : 0;
            const int pj = j1 < n ? sc.p[j1c] : -1;
            if (pj < 0) {
                jend = j1 < n ? j1 : -1;   // no candidate: non-finite costs
                dend = dmin;
                break;
            }
            for (int s = 0; s < K; ++s) used[s] = used[s] || (c[s] == j1);
            j0 = j1;
            i0 = pj;
            ui0 = sc.ut[j1c];
            d0 = dmin;
        }
        // Dual shift of the scanned tree; predecessors published for the flip.
        for (int s = 0; s < K; ++s) {
            if (ok[s] && used[s]) {
                const T sh = dend - dist[s];
                v[s] -= sh;
                ucol[s] += sh;
            }
            if (!ok[s]) continue;
            sc.way[c[s]] = way[s];
            sc.ut[c[s]] = ucol[s];
        }
        wave_sync();
        // Flip the path: every column on it takes the row (and row dual) of
        // its predecessor column; the first one takes the new row.  Columns on
        // the path are found by walking the predecessors from the end; every
        // lane walks (the same) path and updates the columns it holds, reading
        // the old rows and duals from LDS.
        int newp[K];
        T newu[K];
        for (int s = 0; s < K; ++s) {
            newp[s] = p[s];
            newu[s] = ucol[s];
        }
        for (int j = jend, hop = 0; j >= 0 && j < n && hop <= n; ++hop) {
            const int w = sc.way[j];
            const int wc = w >= 0 ? w : 0;
            const int pw = sc.p[wc];
            const T uw = sc.ut[wc];
            for (int s = 0; s < K; ++s) {
                if (c[s] == j) {
                    newp[s] = w >= 0 ? pw : i;
                    newu[s] = w >= 0 ? uw : ufree + dend;
                }
            }
            j = w;
        }
        wave_sync();
        for (int s = 0; s < K; ++s) {
            p[s] = newp[s];
            ucol[s] = newu[s];
            if (!ok[s]) continue;
            sc.p[c[s]] = p[s];
            sc.ut[c[s]] = ucol[s];
        }
        wave_sync();
    }

    return lap_canonical_finish<T, SEG, K, DOWN>(sc, n, R, ldr, duals, assign, v, p, ucol);
}

// Lane bits of a predicate over this lane's segment (bit 0 = the segment's
// first lane), and the lowest set bit (-1 when none).
template <int SEG>
struct SegBits {
    __device__ __forceinline__ static unsigned long long get(bool pred) {
        const unsigned long long b = ballot64(pred);
        if constexpr (SEG == 64)
            return b;
        else
            return (b >> (threadIdx.x & (64 - SEG))) & ((1ull << SEG) - 1);
    }
    // This lane's segment's bits of a wave mask.
    __device__ __forceinline__ static unsigned long long seg(unsigned long long b) {
        if constexpr (SEG == 64)
            return b;
        else
            return (b >> (threadIdx.x & (64 - SEG))) & ((1ull << SEG) - 1);
    }
    __device__ __forceinline__ static int first(unsigned long long bits) {
        if constexpr (SEG == 64)
            return bits ? __builtin_ctzll(bits) : -1;
        else
            return bits ? __builtin_ctz((unsigned)bits) : -1;
    }
};

// The two canonical passes of lap_canonical_finish side by side, for one
// column per lane (n <= SEG, SEG >= 16): the first SEG/2 lanes of a segment
// run the column pass and the other SEG/2 the row pass, each lane holding
// nodes h and h + SEG/2, so both take n steps together.  A relaxation is
// written (M - per-step dual) - per-node dual for both passes.  A fixed node
// keeps its label (it is never relaxed again) and is masked out of the
// minimum; the lowest node at the minimum is the minimum over the lanes of
// their lowest candidate index.  On return (lane as column / as row, K = 1
// layout) vc is the column-canonical dual of the lane's column, ur the
// row-canonical dual of its row and sg its row's column.  Expects sc.p
// (offset r*ld of the row matched to each column) and sc.ut (that row's dual);
// poff is this lane's.
template <typename T, int SEG>
__device__ __forceinline__ void canonical_split(const SlotScratch<T, SEG, 1>& sc, int n, T v, int poff, T& vc,
                                                T& ur, int& sg)
{
    static_assert(SEG >= 16, "two half segments of at least 8 lanes");
    constexpr int H = SEG / 2;
    constexpr int NONE = 1 << 20;
    using HS = SegS<H>;
    const T* __restrict__ M = sc.M;
    const int ldm = sc.ld;   // row stride of M
    const int l = threadIdx.x & (SEG - 1);
    const T INF = inf_of<T>();
    // sigma (column of each row) and v in LDS; sigma also as 16-bit keys in
    // sc.way, right after the column pass's keys sc.p (the row offsets), so
    // both passes read their key with one load.  prow = poff / ld: poff = r ld
    // with r < 64, and the reciprocal's relative error (a few 2^-24) moves
    // r by far less than 1/2.
    const int prow = poff >= 0 ? (int)__builtin_rintf((float)poff * __builtin_amdgcn_rcpf((float)ldm)) : -1;
    if (l < n && prow >= 0 && prow < n) {
        sc.aux[prow] = l;
        sc.way[prow] = (short)l;
    }
    if (l < n) sc.vt[l] = v;
    wave_sync();
    const bool rowpass = l >= H;
    const short* __restrict__ keys = rowpass ? sc.way : sc.p;
    const int h = l & (H - 1);
    int t[2], base[2];
    T lab[2], w[2];
    unsigned long long fxm[2];   // fixed (or absent) node, as wave masks
    for (int q = 0; q < 2; ++q) {
        t[q] = h + q * H;
        const bool okn = t[q] < n;
        const int tc = okn ? t[q] : 0;
        if (rowpass) {
            int sgt = sc.aux[tc];
            sgt = (sgt >= 0 && sgt < n) ? sgt : 0;
            w[q] = sc.ut[sgt];       // u_r of row t: the dual stored at its column
        } else {
            w[q] = sc.vt[tc];       // v_q
        }
        lab[q] = okn ? -w[q] : (T)0;
        fxm[q] = ballot64(!okn);
        // M entry of node t relaxed through a fixed node with key K (column
        // pass: K = offset of p(f); row pass: K = sigma(f)) is M[base + K].
        base[q] = rowpass ? tc * ldm : tc;
    }
    // Every segment takes the wave's largest n steps, so the loop counter is
    // scalar: a segment past its own n has every node fixed, and its further
    // steps (with key 0) change no label.  The steps are branch-free: every
    // node's relaxation is computed (the entry read for a fixed or absent node
    // is in range and its result is discarded).
    int nw = 0;
#pragma unroll
    for (int g = 0; g < 64 / SEG; ++g) nw = ::max(nw, __builtin_amdgcn_readlane(n, g * SEG));
    for (int step = 0; step < nw; ++step) {
        const bool fx0 = lane_bit(fxm[0]), fx1 = lane_bit(fxm[1]);
        const T dmin = HS::min(tmin(fx0 ? INF : lab[0], fx1 ? INF : lab[1]));
        const int cand = (!fx0 && lab[0] == dmin) ? t[0] : ((!fx1 && lab[1] == dmin) ? t[1] : NONE);
        const int f = HS::imin(cand);
        const bool fin = f < n;
        const int fc = fin ? f : 0;
        const int kf = keys[fc];
        const int key = fin ? kf : 0;
        const T s1 = rowpass ? sc.vt[key] : sc.ut[fc];
        for (int q = 0; q < 2; ++q) {
            fxm[q] |= ballot64(t[q] == f);
            const T nd = dmin + ((M[base[q] + key] - s1) - w[q]);
            lab[q] = (!lane_bit(fxm[q]) && nd < lab[q]) ? nd : lab[q];
        }
    }
    wave_sync();
    // Column pass: v^c = v + x into vb; row pass: u^r = u + y into u (the
    // solver's duals are no longer needed).
    for (int q = 0; q < 2; ++q) {
        if (t[q] < n) {
            if (rowpass)
                sc.ut[t[q]] = w[q] + lab[q];
            else
                sc.vt[t[q]] = w[q] + lab[q];
        }
    }
    wave_sync();
    const int lc = l < n ? l : 0;
    vc = sc.vt[lc];
    ur = sc.ut[lc];
    sg = sc.aux[lc];
    wave_sync();
}

// Same contract as lap_concentrate_slots, for one column per lane (n <= SEG),
// with the free rows of all the wave's problems inserted in one loop: each
// pass, every segment that still has a free row takes one Dijkstra step, and a
// segment whose step reached an unmatched column augments and starts on its
// next free row while the others go on, so a wave runs as many passes as its
// busiest problem needs rather than the sum over rows of the busiest problem
// per row.  The argmin is a ballot of the lanes at the minimum (the lowest
// such lane is the lowest column), and the matched rows are kept in LDS as row
// offsets r * ld.  The decisions and the arithmetic are those of
// lap_concentrate_slots.
template <typename T, int SEG, bool DOWN>
__device__ __forceinline__ double lap_concentrate_flat(const SlotScratch<T, SEG, 1>& sc, int n,
                                                       T* __restrict__ R, long long ldr, T* __restrict__ duals,
                                                       int32_t* __restrict__ assign)
{
    using S = SegS<SEG>;
    using Bits = SegBits<SEG>;
    const T* __restrict__ M = sc.M;
    const int ldm = sc.ld;   // row stride of M
    const int l = S::lane();
    const bool ok = l < n;
    const T INF = inf_of<T>();

    // ---- two-sided reduction and greedy start -------------------------------
    T v;
    int poff;   // offset r * ld of the matched row, -1 when free
    T ucol;     // dual of that row
    unsigned long long freem;   // free rows (bit r)
    {
        const int cl[1] = {l};
        const bool okl[1] = {ok};
        T va[1];
        int rw[1];
        const unsigned long long taken = lap_reduce_start<T, SEG, 1>(sc, n, cl, okl, va, rw);
        v = va[0];
        poff = rw[0] >= 0 ? __umul24(rw[0], ldm) : -1;
        ucol = rw[0] >= 0 ? sc.vt[rw[0]] : (T)0;
        if (ok) {
            sc.p[l] = poff;
            sc.ut[l] = ucol;
        }
        freem = ~taken & (n >= 64 ? ~0ull : ((1ull << n) - 1ull));
    }
    wave_sync();

    // ---- Hungarian method, all problems of the wave together -----------------
    int row = Bits::first(freem);   // free row being inserted, -1 when done
    freem &= freem - 1;
    T dist = INF;
    int way = -1;
    int i0n = row >= 0 ? __umul24(row, ldm) : 0;   // offset of the row being scanned
    T urow0 = row >= 0 ? sc.vt[row] : (T)0;   // dual of the free row being inserted
    T ui0 = urow0;                                // dual of the row being scanned
    T d0 = 0;
    int j0 = -1;
    // Lane predicates as wave masks: the columns in range, the columns
    // already in their problem's shortest-path tree, the lanes of problems
    // still inserting a row.
    const unsigned long long okm = ballot64(ok);
    unsigned long long usedm = 0;
    for (;;) {
        const unsigned long long actm = ballot64(row >= 0);
        if (actm == 0) break;
        const unsigned long long livem = actm & okm & ~usedm;
        const bool live = lane_bit(livem);
        const T cur = d0 + ((M[i0n + (ok ? l : 0)] - ui0) - v);
        const bool better = live && cur < dist;
        dist = better ? cur : dist;
        way = better ? j0 : way;
        const T lm = live ? dist : INF;
        const T dmin = S::min(lm);
        const int j1 = Bits::first(Bits::seg(ballot64(lm == dmin) & livem));
        const int jc = j1 >= 0 ? j1 : 0;
        const int pj = sc.p[jc];
        const T uj = sc.ut[jc];
        // Problems whose step reached an unmatched column (or no column).
        const unsigned long long augm = actm & (ballot64(j1 < 0) | ballot64(pj < 0));
        usedm |= ballot64(l == j1);
        j0 = j1;
        i0n = pj >= 0 ? pj : 0;
        ui0 = uj;
        d0 = dmin;
        if (augm != 0) {
            const bool aug = lane_bit(augm);
            const bool used = lane_bit(usedm);
            // Dual shift of the scanned tree (the reached column has dist =
            // dmin, so its shift is 0), predecessors published for the flip.
            if (aug) {
                if (used) {
                    const T sh = dmin - dist;
                    v -= sh;
                    ucol += sh;
                }
                if (ok) {
                    sc.way[l] = way;
                    sc.ut[l] = ucol;
                }
            }
            wave_sync();
            // Flip the path from the reached column back to the new row: a
            // column on it takes the row and row dual of its predecessor (read
            // by every lane at once), the first one the new row.  Only the
            // walk that marks the path is serial.
            int newp = poff;
            T newu = ucol;
            if (aug) {
                const int wc = way >= 0 ? way : 0;
                const int pw = sc.p[wc];
                const T uw = sc.ut[wc];
                bool onpath = false;
                for (int j = j1, hop = 0; j >= 0 && hop <= n; ++hop) {
                    onpath = onpath || (l == j);
                    j = sc.way[j];
                }
                if (onpath) {
                    newp = way >= 0 ? pw : __umul24(row, ldm);
                    newu = way >= 0 ? uw : urow0 + dmin;
                }
            }
            wave_sync();
            if (aug) {
                poff = newp;
                ucol = newu;
                if (ok) {
                    sc.p[l] = poff;
                    sc.ut[l] = ucol;
                }
                row = Bits::first(freem);
                freem &= freem - 1;
                dist = INF;
                way = -1;
                i0n = row >= 0 ? __umul24(row, ldm) : 0;
                urow0 = row >= 0 ? sc.vt[row] : (T)0;
                ui0 = urow0;
                d0 = 0;
                j0 = -1;
            }
            usedm &= ~augm;   // the new rows start with empty trees
            wave_sync();
        }
    }

    if constexpr (SEG >= 16) {
        T vc, ur;
        int sg;
        canonical_split<T, SEG>(sc, n, v, poff, vc, ur, sg);
        const T vca[1] = {vc};
        const T ura[1] = {ur};
        const int sga[1] = {sg};
        return lap_complete<T, SEG, 1, DOWN>(sc, n, R, ldr, duals, assign, vca, ura, sga);
    } else {
        // Row indices for the sequential canonical passes.
        const int prow = poff >= 0 ? poff / ldm : -1;
        if (ok) sc.p[l] = prow;
        wave_sync();
        const T va[1] = {v};
        const int pa[1] = {prow};
        const T ua[1] = {ucol};
        return lap_canonical_finish<T, SEG, 1, DOWN>(sc, n, R, ldr, duals, assign, va, pa, ua);
    }
}

// canonical_split for K columns per lane (n <= SEG * K, SEG >= 16): the two
// half segments of SEG/2 lanes run the column and the row pass side by side,
// each lane holding the 2K nodes h, h + SEG/2, ..., h + (2K-1) SEG/2.  Same
// decisions and operations as canonical_split (and lap_canonical_finish):
// the lowest node at the minimum, relaxations (M - per-step dual) - per-node
// dual.  poff[s] is the offset r*ld of the row matched to column c_s (-1 when
// none); on return vc, ur and sg hold, for each of the lane's columns c_s
// (rows c_s), the column-canonical dual, the row-canonical dual and the
// row's column.
template <typename T, int SEG, int K>
__device__ __forceinline__ void canonical_split_k(const SlotScratch<T, SEG, K>& sc, int n, const T (&v)[K],
                                                  const int (&poff)[K], T (&vc)[K], T (&ur)[K], int (&sg)[K])
{
    static_assert(SEG >= 16, "two half segments of at least 8 lanes");
    constexpr int H = SEG / 2;
    constexpr int NQ = 2 * K;
    constexpr int NONE = 1 << 20;
    using HS = SegS<H>;
    const T* __restrict__ M = sc.M;
    const int ldm = sc.ld;   // row stride of M
    const int l = threadIdx.x & (SEG - 1);
    const T INF = inf_of<T>();
    for (int s = 0; s < K; ++s) {
        const int c = s * SEG + l;
        if (c >= n) continue;
        const int prow = poff[s] >= 0 ? (int)__builtin_rintf((float)poff[s] * __builtin_amdgcn_rcpf((float)ldm)) : -1;
        if (prow >= 0 && prow < n) {
            sc.aux[prow] = c;
            sc.way[prow] = (short)c;
        }
        sc.vt[c] = v[s];
    }
    wave_sync();
    const bool rowpass = l >= H;
    const short* __restrict__ keys = rowpass ? sc.way : sc.p;
    const int h = l & (H - 1);
    int t[NQ], base[NQ];
    T lab[NQ], w[NQ];
    bool fx[NQ];
    for (int q = 0; q < NQ; ++q) {
        t[q] = h + q * H;
        const bool okn = t[q] < n;
        const int tc = okn ? t[q] : 0;
        if (rowpass) {
            int sgt = sc.aux[tc];
            sgt = (sgt >= 0 && sgt < n) ? sgt : 0;
            w[q] = sc.ut[sgt];
        } else {
            w[q] = sc.vt[tc];
        }
        lab[q] = okn ? -w[q] : (T)0;
        fx[q] = !okn;
        base[q] = rowpass ? tc * ldm : tc;
    }
    for (int step = 0; step < n; ++step) {
        T m = fx[0] ? INF : lab[0];
        for (int q = 1; q < NQ; ++q) m = tmin(m, fx[q] ? INF : lab[q]);
        const T dmin = HS::min(m);
        int cand = NONE;
        for (int q = NQ - 1; q >= 0; --q)
            if (!fx[q] && lab[q] == dmin) cand = t[q];
        const int f = HS::imin(cand);
        const int fc = f < n ? f : 0;
        const int key = keys[fc];
        const T s1 = rowpass ? sc.vt[key] : sc.ut[fc];
        for (int q = 0; q < NQ; ++q) {
            fx[q] = fx[q] || (t[q] == f);
            const T nd = dmin + ((M[base[q] + key] - s1) - w[q]);
            lab[q] = (!fx[q] && nd < lab[q]) ? nd : lab[q];
        }
    }
    wave_sync();
    for (int q = 0; q < NQ; ++q) {
        if (t[q] < n) {
            if (rowpass)
                sc.ut[t[q]] = w[q] + lab[q];
            else
                sc.vt[t[q]] = w[q] + lab[q];
        }
    }
    wave_sync();
    for (int s = 0; s < K; ++s) {
        const int c = s * SEG + l;
        const int cc = c < n ? c : 0;
        vc[s] = sc.vt[cc];
        ur[s] = sc.ut[cc];
        sg[s] = sc.aux[cc];
    }
    wave_sync();
}

// lap_concentrate_flat for K columns per lane (n <= SEG * K, SEG >= 16):
// the free rows of all the wave's problems inserted in one loop, each lane
// holding columns c_s = s*SEG + lane.  Per Dijkstra step every lane scans its
// K columns, the segment minimum runs over the lanes' smallest, and the
// lowest column at the minimum is the lowest lane of the lowest slot whose
// ballot is not empty.  Same decisions and arithmetic as
// lap_concentrate_slots.
template <typename T, int SEG, int K, bool DOWN>
__device__ __forceinline__ double lap_concentrate_flatk(const SlotScratch<T, SEG, K>& sc, int n,
                                                        T* __restrict__ R, long long ldr, T* __restrict__ duals,
                                                        int32_t* __restrict__ assign)
{
    static_assert(SEG >= 16 && K >= 2, "several columns per lane, half segments of at least 8 lanes");
    using S = SegS<SEG>;
    using Bits = SegBits<SEG>;
    const T* __restrict__ M = sc.M;
    const int ldm = sc.ld;   // row stride of M
    const int l = S::lane();
    const T INF = inf_of<T>();
    int c[K];
    bool ok[K];
    for (int s = 0; s < K; ++s) {
        c[s] = s * SEG + l;
        ok[s] = c[s] < n;
    }

    // ---- two-sided reduction and greedy start -------------------------------
    T v[K];
    int poff[K];   // offset r * ld of the row matched to each column, -1 when free
    T ucol[K];     // dual of that row
    unsigned long long freem;
    {
        int rw[K];
        const unsigned long long taken = lap_reduce_start<T, SEG, K>(sc, n, c, ok, v, rw);
        for (int s = 0; s < K; ++s) {
            poff[s] = rw[s] >= 0 ? __umul24(rw[s], ldm) : -1;
            ucol[s] = rw[s] >= 0 ? sc.vt[rw[s]] : (T)0;
        }
        freem = ~taken & (n >= 64 ? ~0ull : ((1ull << n) - 1ull));
    }
    wave_sync();
    for (int s = 0; s < K; ++s) {
        if (!ok[s]) continue;
        sc.p[c[s]] = poff[s];
        sc.ut[c[s]] = ucol[s];
    }
    wave_sync();

    // ---- Hungarian method, all problems of the wave together -----------------
    int row = freem ? __builtin_ctzll(freem) : -1;
    freem &= freem - 1;
    T dist[K];
    int way[K];
    bool used[K];
    for (int s = 0; s < K; ++s) {
        dist[s] = INF;
        way[s] = -1;
        used[s] = false;
    }
    int i0n = row >= 0 ? __umul24(row, ldm) : 0;
    T urow0 = row >= 0 ? sc.vt[row] : (T)0;
    T ui0 = urow0;
    T d0 = 0;
    int j0 = -1;
    while (ballot64(row >= 0) != 0) {
        const bool active = row >= 0;
        bool live[K];
        T lm[K];
        for (int s = 0; s < K; ++s) {
            live[s] = active && ok[s] && !used[s];
            const T cur = d0 + ((M[i0n + (ok[s] ? c[s] : 0)] - ui0) - v[s]);
            const bool better = live[s] && cur < dist[s];
            dist[s] = better ? cur : dist[s];
            way[s] = better ? j0 : way[s];
            lm[s] = live[s] ? dist[s] : INF;
        }
        T lmin = lm[0];
        for (int s = 1; s < K; ++s) lmin = tmin(lmin, lm[s]);
        const T dmin = S::min(lmin);
        int j1 = -1;
        for (int s = 0; s < K; ++s) {
            const unsigned long long bs = Bits::get(live[s] && lm[s] == dmin);
            if (j1 < 0 && bs != 0ull) j1 = s * SEG + Bits::first(bs);
        }
        const int jc = j1 >= 0 ? j1 : 0;
        const int pj = sc.p[jc];
        const T uj = sc.ut[jc];
        const bool aug = active && (j1 < 0 || pj < 0);
        for (int s = 0; s < K; ++s) used[s] = used[s] || (c[s] == j1);
        j0 = j1;
        i0n = pj >= 0 ? pj : 0;
        ui0 = uj;
        d0 = dmin;
        if (ballot64(aug) != 0) {
            if (aug) {
                for (int s = 0; s < K; ++s) {
                    if (used[s]) {
                        const T sh = dmin - dist[s];
                        v[s] -= sh;
                        ucol[s] += sh;
                    }
                    if (ok[s]) {
                        sc.way[c[s]] = way[s];
                        sc.ut[c[s]] = ucol[s];
                    }
                }
            }
            wave_sync();
            int newp[K];
            T newu[K];
            for (int s = 0; s < K; ++s) {
                newp[s] = poff[s];
                newu[s] = ucol[s];
            }
            if (aug) {
                bool onpath[K];
                for (int s = 0; s < K; ++s) onpath[s] = false;
                for (int j = j1, hop = 0; j >= 0 && hop <= n; ++hop) {
                    for (int s = 0; s < K; ++s) onpath[s] = onpath[s] || (c[s] == j);
                    j = sc.way[j];
                }
                for (int s = 0; s < K; ++s) {
                    if (!onpath[s]) continue;
                    const int wc = way[s] >= 0 ? way[s] : 0;
                    newp[s] = way[s] >= 0 ? (int)sc.p[wc] : __umul24(row, ldm);
                    newu[s] = way[s] >= 0 ? sc.ut[wc] : urow0 + dmin;
                }
            }
            wave_sync();
            if (aug) {
                for (int s = 0; s < K; ++s) {
                    poff[s] = newp[s];
                    ucol[s] = newu[s];
                    if (ok[s]) {
                        sc.p[c[s]] = poff[s];
                        sc.ut[c[s]] = ucol[s];
                    }
                    dist[s] = INF;
                    way[s] = -1;
                    used[s] = false;
                }
                row = freem ? __builtin_ctzll(freem) : -1;
                freem &= freem - 1;
                i0n = row >= 0 ? __umul24(row, ldm) : 0;
                urow0 = row >= 0 ? sc.vt[row] : (T)0;
                ui0 = urow0;
                d0 = 0;
                j0 = -1;
            }
            wave_sync();
        }
    }

    T vc[K], ur[K];
    int sg[K];
    canonical_split_k<T, SEG, K>(sc, n, v, poff, vc, ur, sg);
    return lap_complete<T, SEG, K, DOWN>(sc, n, R, ldr, duals, assign, vc, ur, sg);
}

}  // namespace qap
