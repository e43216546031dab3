// Wavefront-level linear assignment with canonical dual, for gfx950 (wave64).
//
// Cost concentration (Section 4.1 of arXiv 1510.02065) solves one assignment
// problem per block of the reduced-cost array, moves its value S to the parent
// coefficient and replaces the block by its residuals.  Here a "segment" of
// SEG lanes (SEG in {8,16,32,64}, SEG >= n) owns one n x n problem whose
// matrix sits in LDS; lane j stands for column j and, where noted, for row j.
// A wave therefore works on 64/SEG problems at once.
//
// Solver: the Hungarian method in its shortest-augmenting-path form (Munkres;
// rows inserted one at a time, Dijkstra over columns on reduced costs).  Each
// Dijkstra step is one LDS row read per lane plus a segment-wide argmin.
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
// column; one dense Dijkstra pass computes it.  The row point is the same on
// the row graph.  Both residual halves are >= 0 exactly: the subtracted dual
// is a row (column) minimum of the already rounded differences.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qap {

template <typename T> __device__ __forceinline__ T inf_of();
template <> __device__ __forceinline__ double inf_of<double>() { return __builtin_huge_val(); }
template <> __device__ __forceinline__ float inf_of<float>() { return __builtin_huge_valf(); }

// Segment-wide collectives.  All lanes of a segment must be active when one of
// these is called; segments of the same wave are independent.
template <int SEG>
struct Seg {
    static_assert(SEG == 8 || SEG == 16 || SEG == 32 || SEG == 64, "segment size");
    __device__ __forceinline__ static int lane() { return threadIdx.x & (SEG - 1); }
    __device__ __forceinline__ static int base() { return (threadIdx.x & 63) & ~(SEG - 1); }

    // min over the segment; every lane receives the same value.
    template <typename T>
    __device__ __forceinline__ static T min(T x) {
#pragma unroll
        for (int m = 1; m < SEG; m <<= 1) {
            T y = __shfl_xor(x, m, 64);
            x = (y < x) ? y : x;
        }
        return x;
    }
    // sum over the segment by a butterfly; addition is commutative, so every
    // lane receives bitwise the same value.
    template <typename T>
    __device__ __forceinline__ static T sum(T x) {
#pragma unroll
        for (int m = 1; m < SEG; m <<= 1) x = x + __shfl_xor(x, m, 64);
        return x;
    }
    // lowest segment lane with pred true (SEG if none).
    __device__ __forceinline__ static int first(bool pred) {
        unsigned long long m = __ballot(pred);
        unsigned long long s = (SEG == 64) ? m : ((m >> base()) & ((1ull << SEG) - 1ull));
        return s ? (int)__builtin_ctzll(s) : SEG;
    }
    // value of x held by segment lane src (src may differ per lane).
    template <typename T>
    __device__ __forceinline__ static T read(T x, int src) { return __shfl(x, base() + src, 64); }
};

// Per-segment LDS working set, laid out as [matrix n*n | sig SEG | vecA SEG | vecB SEG].
template <typename T, int SEG>
struct SegLds {
    __host__ __device__ static size_t bytes(int n) {
        size_t m = (size_t)n * n * sizeof(T);
        m = (m + 15) & ~(size_t)15;
        return m + SEG * (sizeof(int) + 2 * sizeof(T));
    }
};

// Solve, canonicalise and write residuals for the n x n matrix M (in LDS).
//   n        problem size for this segment (0 <= n <= SEG; segment-uniform).
//   M        segment's LDS matrix, row stride n (left unchanged).
//   sig_s, va_s, vb_s: segment's LDS scratch (SEG entries each).
//   R        nullable; receives the residual, row stride n (global memory).
//   duals    nullable; receives [uc | vc | ur | vr] (4n values).
//   assign   nullable; assign[r] = column of row r in the solver's assignment.
// Returns S to every lane of the segment.  Must be called by whole waves in
// uniform control flow (it contains block barriers; launch one wave per
// workgroup).
template <typename T, int SEG>
__device__ double lap_concentrate_seg(const T* __restrict__ M, int n, int* __restrict__ sig_s,
                                      T* __restrict__ va_s, T* __restrict__ vb_s,
                                      T* __restrict__ R, T* __restrict__ duals,
                                      int32_t* __restrict__ assign)
{
    using S = Seg<SEG>;
    const int lane = S::lane();
    const bool ok = lane < n;
    const T INF = inf_of<T>();

    // ---- Hungarian method, shortest augmenting paths -----------------------
    // Column lane j keeps: v (column dual), p (row matched to column j or -1),
    // ucol (dual of row p).  The row being inserted has dual ufree.
    T v = 0, ucol = 0;
    int p = -1;
    for (int i = 0; i < n; ++i) {
        T minv = INF;   // tentative reduced distance to column j
        int way = -1;   // previous column on the shortest path (-1: the new row)
        bool used = false;
        T ufree = 0;
        int i0 = i;     // row being scanned
        T ui0 = 0;      // its dual
        int j0 = -1;    // column through which row i0 was reached
        int jend = -1;
        // Each pass marks one more column as scanned, so a well-formed search
        // ends within n passes; the bound also ends it on non-finite input.
        for (int pass = 0; pass <= n; ++pass) {
            if (ok && !used) {
                T cur = (M[i0 * n + lane] - ui0) - v;
                if (cur < minv) {
                    minv = cur;
                    way = j0;
                }
            }
            const T cand = (ok && !used) ? minv : INF;
            const T delta = S::min(cand);
            const int j1 = S::first(ok && !used && cand == delta);
            if (j1 >= n) break;   // no candidate: non-finite costs
            if (ok) {
                if (used) {
                    v -= delta;
                    ucol += delta;
                } else {
                    minv -= delta;
                }
            }
            ufree += delta;
            const int pj = S::read(p, j1);
            const T uj = S::read(ucol, j1);
            if (pj < 0) {
                jend = j1;
                break;
            }
            if (lane == j1) used = true;
            j0 = j1;
            i0 = pj;
            ui0 = uj;
        }
        // Flip the path: every column on it takes the row (and row dual) of
        // its predecessor column; the first one takes the new row.
        bool onpath = false;
        for (int j = jend, hop = 0; j >= 0 && j < n && hop <= n; ++hop) {
            if (lane == j) onpath = true;
            j = S::read(way, j);
        }
        const int src = (way >= 0) ? way : lane;
        const int pw = S::read(p, src);
        const T uw = S::read(ucol, src);
        if (onpath) {
            p = (way >= 0) ? pw : i;
            ucol = (way >= 0) ? uw : ufree;
        }
    }

    // sigma (column of row r) for lane r, and the solver's row dual u_r.
    if (ok && p >= 0 && p < n) sig_s[p] = lane;
    __syncthreads();
    const int sig = ok ? sig_s[lane] : 0;
    const T urow = S::read(ucol, sig);

    // ---- column-canonical point (lanes = columns) ---------------------------
    T dist = ok ? -v : INF;
    bool done = !ok;
    for (int s = 0; s < n; ++s) {
        const T cand = done ? INF : dist;
        const T dmin = S::min(cand);
        const int c = S::first(!done && cand == dmin);
        if (c >= n) break;
        const int r = S::read(p, c);
        const T ur = S::read(ucol, c);
        if (lane == c) done = true;
        if (!done) {
            const T nd = dmin + ((M[r * n + lane] - ur) - v);
            if (nd < dist) dist = nd;
        }
    }
    const T vc = v + dist;
    if (ok) va_s[lane] = vc;
    __syncthreads();
    T uc = INF;   // lane as row r
    if (ok) {
        for (int q = 0; q < n; ++q) {
            const T t = M[lane * n + q] - va_s[q];
            uc = (t < uc) ? t : uc;
        }
    }

    // ---- row-canonical point (lanes = rows) ---------------------------------
    T distr = ok ? -urow : INF;
    bool doner = !ok;
    for (int s = 0; s < n; ++s) {
        const T cand = doner ? INF : distr;
        const T dmin = S::min(cand);
        const int srow = S::first(!doner && cand == dmin);
        if (srow >= n) break;
        const int cs = S::read(sig, srow);
        const T vcs = S::read(v, cs);
        if (lane == srow) doner = true;
        if (!doner) {
            const T nd = dmin + ((M[lane * n + cs] - urow) - vcs);
            if (nd < distr) distr = nd;
        }
    }
    const T ur = urow + distr;
    __syncthreads();
    if (ok) vb_s[lane] = ur;
    __syncthreads();
    T vr = INF;   // lane as column q
    if (ok) {
        for (int r = 0; r < n; ++r) {
            const T t = M[r * n + lane] - vb_s[r];
            vr = (t < vr) ? t : vr;
        }
    }
    __syncthreads();
    if (ok) va_s[lane] = uc;
    __syncthreads();

    // ---- residual and transferred value -------------------------------------
    if (R != nullptr && ok) {
        for (int r = 0; r < n; ++r) {
            const T m = M[r * n + lane];
            const T r1 = (m - vc) - va_s[r];
            const T r2 = (m - vb_s[r]) - vr;
            R[r * n + lane] = (T)0.5 * (r1 + r2);
        }
    }
    if (duals != nullptr && ok) {
        duals[lane] = uc;
        duals[n + lane] = vc;
        duals[2 * n + lane] = ur;
        duals[3 * n + lane] = vr;
    }
    if (assign != nullptr && ok) assign[lane] = sig;

    const T suc = S::sum(ok ? uc : (T)0);
    const T svc = S::sum(ok ? vc : (T)0);
    const T sur = S::sum(ok ? ur : (T)0);
    const T svr = S::sum(ok ? vr : (T)0);
    __syncthreads();
    return 0.5 * ((double)(suc + svc) + (double)(sur + svr));
}

}  // namespace qap
