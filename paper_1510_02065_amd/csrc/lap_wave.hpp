// Wavefront-level linear assignment with canonical dual, for gfx950 (wave64).
//
// Cost concentration (Section 4.1 of arXiv 1510.02065) solves one assignment
// problem per block of the reduced-cost array, moves its value S to the parent
// coefficient and replaces the block by its residuals.  Here a "segment" of
// SEG lanes (SEG in {8,16,32,64}, SEG >= n) owns one n x n problem whose
// matrix sits in LDS; lane j stands for column j and, where noted, for row j.
// A wave therefore works on 64/SEG problems at once.
//
// Solver: the Hungarian method in its shortest-augmenting-path form (Munkres),
// started from the Jonker-Volgenant column reduction: v_j is the minimum of
// column j and each row that is the first minimum of some column is matched to
// the lowest such column.  The remaining free rows are inserted one at a time
// by Dijkstra over columns on reduced costs; each Dijkstra step is one LDS row
// read per lane plus a segment-wide argmin.
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
// column.  One dense Dijkstra pass over the columns computes it.  The row
// point is the same on the row graph.  Both
// residual halves are >= 0 exactly: the subtracted dual is a row (column)
// minimum of the already rounded differences.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlt2_kernels.hpp"

namespace qap {

// Wave-wide ballot of a predicate; taking a bool (not an int as __ballot
// does) lets the compiler use the comparison's lane mask directly.
__device__ __forceinline__ unsigned long long ballot64(bool pred) { return __builtin_amdgcn_ballot_w64(pred); }

template <typename T> __device__ __forceinline__ T inf_of();
template <> __device__ __forceinline__ double inf_of<double>() { return __builtin_huge_val(); }
template <> __device__ __forceinline__ float inf_of<float>() { return __builtin_huge_valf(); }

// ---- cross-lane primitives ---------------------------------------------------
// Reductions use no LDS.  DPP controls (gfx9 encoding): quad_perm(1,0,3,2)
// pairs lane^1, quad_perm(2,3,0,1) pairs lane^2, row_half_mirror reverses 8
// lanes and row_mirror 16 lanes.  After the two quad swaps every lane of a
// quad holds the quad's value; each mirror then combines a group with its
// neighbour, so the four steps all-reduce 16 lanes.  permlane16_swap and
// permlane32_swap (gfx950) called with the same register twice return, in
// their two results, the lane's own value and the value 16 (32) lanes away in
// some order, which is all a commutative reduction needs.
enum : int { kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140 };

template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) { return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true); }
template <int CTRL>
__device__ __forceinline__ float dpp(float x) { return __int_as_float(dpp_i<CTRL>(__float_as_int(x))); }
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
    const int lo = dpp_i<CTRL>(__double2loint(x));
    const int hi = dpp_i<CTRL>(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

template <int HALF>
__device__ __forceinline__ void swap_pair(float x, float& a, float& b) {
    const unsigned u = __float_as_uint(x);
    if constexpr (HALF == 16) {
        auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        a = __uint_as_float(r[0]);
        b = __uint_as_float(r[1]);
    } else {
        auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        a = __uint_as_float(r[0]);
        b = __uint_as_float(r[1]);
    }
}
template <int HALF>
__device__ __forceinline__ void swap_pair(double x, double& a, double& b) {
    const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
    if constexpr (HALF == 16) {
        auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        a = __hiloint2double((int)rh[0], (int)rl[0]);
        b = __hiloint2double((int)rh[1], (int)rl[1]);
    } else {
        auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        a = __hiloint2double((int)rh[0], (int)rl[0]);
        b = __hiloint2double((int)rh[1], (int)rl[1]);
    }
}

// Orders this wave's LDS writes before its later LDS reads by other lanes.
// A wave's LDS operations execute in order, so only compiler reordering has to
// be prevented; each wave owns its LDS region, so waves of a workgroup need
// not wait for each other.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float tmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double tmin(double a, double b) { return __builtin_fmin(a, b); }

// Segment-wide collectives for segments of SEG lanes (LPW = 64/SEG segments
// per wave).  All lanes of a segment must be active when one is called;
// segments are independent of each other.
template <int SEG>
struct Seg {
    static_assert(SEG == 8 || SEG == 16 || SEG == 32 || SEG == 64, "segment size");
    static constexpr int LPW = 64 / SEG;
    __device__ __forceinline__ static int lane() { return threadIdx.x & (SEG - 1); }
    __device__ __forceinline__ static int seg() { return (threadIdx.x & 63) / SEG; }
    __device__ __forceinline__ static int base() { return (threadIdx.x & 63) & ~(SEG - 1); }

    // min over the segment; every lane receives the same value.
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
    // sum over the segment by a butterfly; addition is commutative, so every
    // lane receives bitwise the same value.
    template <typename T>
    __device__ __forceinline__ static T sum(T x) {
        x = x + dpp<kDppXor1>(x);
        x = x + dpp<kDppXor2>(x);
        x = x + dpp<kDppHalfMirror>(x);
        if constexpr (SEG >= 16) x = x + dpp<kDppMirror>(x);
        if constexpr (SEG >= 32) {
            T a, b;
            swap_pair<16>(x, a, b);
            x = a + b;
        }
        if constexpr (SEG >= 64) {
            T a, b;
            swap_pair<32>(x, a, b);
            x = a + b;
        }
        return x;
    }

    // sum over the segment with every addition rounded toward -inf; TwoSum
    // is exact and symmetric, so every lane receives the same value.
    __device__ __forceinline__ static double sum_down(double x) {
        x = add_down(x, dpp<kDppXor1>(x));
        x = add_down(x, dpp<kDppXor2>(x));
        x = add_down(x, dpp<kDppHalfMirror>(x));
        if constexpr (SEG >= 16) x = add_down(x, dpp<kDppMirror>(x));
        if constexpr (SEG >= 32) {
            double a, b;
            swap_pair<16>(x, a, b);
            x = add_down(a, b);
        }
        if constexpr (SEG >= 64) {
            double a, b;
            swap_pair<32>(x, a, b);
            x = add_down(a, b);
        }
        return x;
    }

    // Per-segment scalar indices, kept in scalar registers.
    struct Idx {
        int s[LPW];
    };
    // lowest lane of each segment with pred true (SEG if none).
    __device__ __forceinline__ static Idx first(bool pred) {
        const unsigned long long m = ballot64(pred);
        Idx r;
#pragma unroll
        for (int g = 0; g < LPW; ++g) {
            unsigned long long sm = m;
            if constexpr (SEG < 64) sm = (m >> (g * SEG)) & ((1ull << SEG) - 1ull);
            r.s[g] = sm ? (int)__builtin_ctzll(sm) : SEG;
        }
        return r;
    }
    // this lane's segment's entry of a per-segment scalar.
    __device__ __forceinline__ static int mine(const Idx& x) {
        int r = x.s[0];
#pragma unroll
        for (int g = 1; g < LPW; ++g) r = (seg() == g) ? x.s[g] : r;
        return r;
    }
    // value of x at lane idx of each segment, as a per-segment scalar.
    __device__ __forceinline__ static Idx at(int x, const Idx& idx) {
        Idx r;
#pragma unroll
        for (int g = 0; g < LPW; ++g) r.s[g] = __builtin_amdgcn_readlane(x, g * SEG + (idx.s[g] & (SEG - 1)));
        return r;
    }
    // value of x at lane idx of this lane's segment (broadcast by readlane).
    __device__ __forceinline__ static int bcast(int x, const Idx& idx) { return mine(at(x, idx)); }
    __device__ __forceinline__ static float bcast(float x, const Idx& idx) {
        return __int_as_float(bcast(__float_as_int(x), idx));
    }
    __device__ __forceinline__ static double bcast(double x, const Idx& idx) {
        const int lo = bcast(__double2loint(x), idx);
        const int hi = bcast(__double2hiint(x), idx);
        return __hiloint2double(hi, lo);
    }
    // value of x held by segment lane src (src may differ per lane).
    template <typename T>
    __device__ __forceinline__ static T read(T x, int src) { return __shfl(x, base() + src, 64); }
};

// Per-segment LDS working set, laid out as
// [matrix n*n of T | sig: SEG ints | aux: SEG ints | vecA: SEG doubles |
//  vecB: SEG doubles].
template <typename T, int SEG>
struct SegLds {
    __host__ __device__ static size_t mat_bytes(int n) {
        return (((size_t)n * n * sizeof(T)) + 15) & ~(size_t)15;
    }
    __host__ __device__ static size_t bytes(int n) {
        return mat_bytes(n) + SEG * (2 * sizeof(int) + 2 * sizeof(double));
    }
};

// Carves a segment's LDS working set.
template <typename T, int SEG>
struct SegScratch {
    T* M;
    int* sig;
    int* aux;
    double* va;
    double* vb;
    __device__ SegScratch(unsigned char* base, int n) {
        const size_t mb = SegLds<T, SEG>::mat_bytes(n);
        M = reinterpret_cast<T*>(base);
        sig = reinterpret_cast<int*>(base + mb);
        aux = sig + SEG;
        va = reinterpret_cast<double*>(base + mb + 2 * SEG * sizeof(int));
        vb = va + SEG;
    }
};

// Solve, canonicalise and write residuals for the n x n matrix sc.M (in LDS).
//   n        problem size for this segment (0 <= n <= SEG; segment-uniform).
//   sc       segment's LDS working set; sc.M (row stride n) is left unchanged.
//   R        nullable; receives the residual, row stride n (global memory).
//   duals    nullable; receives [uc | vc | ur | vr] (4n values).
//   assign   nullable; assign[r] = column of row r in the solver's assignment.
// Returns S to every lane of the segment.  Must be called by whole waves
// (every segment of the wave, possibly with different n).
template <typename T, int SEG>
__device__ __forceinline__ double lap_concentrate_seg(const SegScratch<T, SEG>& sc, int n,
                                                      T* __restrict__ R, T* __restrict__ duals,
                                                      int32_t* __restrict__ assign)
{
    using S = Seg<SEG>;
    const T* __restrict__ M = sc.M;
    const int lane = S::lane();
    const bool ok = lane < n;
    const int col = ok ? lane : 0;   // clamped column for lanes beyond n
    const T INF = inf_of<T>();
    // During the solve the segment's scratch holds, per column lane j:
    //   sc.sig[j] = p_j (row matched to column j, or -1), sc.va[j] = ucol_j
    // (that row's dual), republished whenever they change, so a Dijkstra step
    // fetches them for the chosen column with two LDS broadcast reads.
    // sc.aux[r] marks rows that are already matched.

    // ---- column reduction -------------------------------------------------
    T v = 0;          // column dual (lane = column)
    int crow = 0;     // first row attaining the column minimum
    if (ok) {
        v = M[lane];
        for (int r = 1; r < n; ++r) {
            const T m = M[r * n + lane];
            if (m < v) {
                v = m;
                crow = r;
            }
        }
    }
    sc.aux[lane] = SEG;
    wave_sync();
    if (ok) atomicMin(&sc.aux[crow], lane);
    wave_sync();
    int p = (ok && sc.aux[crow] == lane) ? crow : -1;
    T ucol = 0;
    sc.sig[lane] = p;
    sc.va[lane] = 0.0;
    wave_sync();

    // ---- Hungarian method for the rows left free -----------------------------
    // Inserting free row i runs Dijkstra over columns with absolute tentative
    // distances `dist` (reduced costs are >= 0); duals are only shifted when
    // the search reaches an unmatched column, by D* - dist_j for every scanned
    // column j (Jonker-Volgenant form).
    for (int i = 0; i < n; ++i) {
        if (sc.aux[i] != SEG) continue;   // row i already matched
        T dist = INF;   // tentative distance from row i to column j
        int way = -1;   // previous column on the shortest path (-1: row i)
        bool used = false;
        int i0 = i;     // row being scanned
        T ui0 = 0;      // its dual (a free row has dual 0)
        T d0 = 0;       // distance at which row i0 was reached
        int j0 = -1;    // column through which row i0 was reached
        int jend = -1;
        T dend = 0;
        // Each pass scans one more column, so a well-formed search ends within
        // n passes; the bound also ends it on non-finite input.
        for (int pass = 0; pass <= n; ++pass) {
            const T cur = d0 + ((M[i0 * n + col] - ui0) - v);
            const bool live = ok && !used;
            if (live && cur < dist) {
                dist = cur;
                way = j0;
            }
            const T cand = live ? dist : INF;
            const T dmin = S::min(cand);
            const int j1 = S::mine(S::first(live && cand == dmin));
            const int j1c = j1 < n ? j1 : 0;
            const int pj = j1 < n ? sc.sig[j1c] : -1;
            if (pj < 0) {
                jend = j1 < n ? j1 : -1;   // no candidate: non-finite costs
                dend = dmin;
                break;
            }
            if (lane == j1) used = true;
            j0 = j1;
            i0 = pj;
            ui0 = (T)sc.va[j1c];
            d0 = dmin;
        }
        // Dual shift of the scanned tree.
        if (ok && used) {
            const T sh = dend - dist;
            v -= sh;
            ucol += sh;
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
            ucol = (way >= 0) ? uw : dend;
        }
        wave_sync();
        sc.sig[lane] = p;
        sc.va[lane] = (double)ucol;
        wave_sync();
    }

    // ---- column-canonical point (lanes = columns) ---------------------------
    // x_q = shortest distance to column q from label -v_q at every column,
    // over arcs c -> q of reduced cost M[p(c)][q] - u_{p(c)} - v_q >= 0.
    T x;
    {
        T dist = ok ? -v : INF;
        bool done = !ok;
        for (int s = 0; s < n; ++s) {
            const T cand = done ? INF : dist;
            const T dmin = S::min(cand);
            const int c = S::mine(S::first(!done && cand == dmin));
            if (c >= n) break;
            const int r = sc.sig[c];
            const T ur = (T)sc.va[c];
            if (lane == c) done = true;
            const T nd = dmin + ((M[r * n + col] - ur) - v);
            if (!done && nd < dist) dist = nd;
        }
        x = ok ? dist : (T)0;
    }

    // sigma (column of row r, lane r) in sc.aux, v in sc.vb; the solver's row
    // dual u_r = ucol at column sigma(r).
    wave_sync();
    if (ok && p >= 0) sc.aux[p] = lane;
    sc.vb[lane] = (double)v;
    wave_sync();
    const int sig = ok ? sc.aux[lane] : 0;
    const T urow = (T)sc.va[sig];

    // ---- row-canonical point (lanes = rows) ---------------------------------
    // y_r = shortest distance to row r from label -u_r at every row, over
    // arcs s -> r of reduced cost M[r][sigma(s)] - u_r - v_{sigma(s)} >= 0.
    T y;
    {
        T dist = ok ? -urow : INF;
        bool done = !ok;
        for (int s = 0; s < n; ++s) {
            const T cand = done ? INF : dist;
            const T dmin = S::min(cand);
            const int srow = S::mine(S::first(!done && cand == dmin));
            if (srow >= n) break;
            const int cs = sc.aux[srow];
            const T vcs = (T)sc.vb[cs];
            if (lane == srow) done = true;
            const T nd = dmin + ((M[col * n + cs] - urow) - vcs);
            if (!done && nd < dist) dist = nd;
        }
        y = ok ? dist : (T)0;
    }
    const T vc = v + x;
    const T ur = urow + y;
    wave_sync();

    if constexpr (sizeof(T) == 8) {
        // ---- FP64: residual = mean of the residuals under the two points ----
        sc.va[lane] = vc;
        sc.vb[lane] = ur;
        wave_sync();
        T uc = INF;   // lane as row r
        T vr = INF;   // lane as column q
        if (ok) {
            for (int q = 0; q < n; ++q) uc = tmin(uc, M[lane * n + q] - (T)sc.va[q]);
            for (int r = 0; r < n; ++r) vr = tmin(vr, M[r * n + lane] - (T)sc.vb[r]);
        }
        wave_sync();
        sc.va[lane] = uc;
        wave_sync();
        if (R != nullptr && ok) {
            for (int r = 0; r < n; ++r) {
                const T m = M[r * n + lane];
                const T r1 = (m - vc) - (T)sc.va[r];
                const T r2 = (m - (T)sc.vb[r]) - vr;
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
        wave_sync();
        return 0.5 * ((suc + svc) + (sur + svr));
    } else {
        // ---- FP32 certified: the duals are completed in FP64 rounding toward
        // -inf, which keeps them feasible (u_r + v_q <= M_rq exactly).  With
        // U = (uc + ur)/2 and V = (vc + vr)/2 the residual M - U - V (the same
        // value as the mean of the two residuals) is then >= 0, and each entry
        // and S = sum U + sum V are rounded down once.
        sc.va[lane] = (double)vc;
        sc.vb[lane] = (double)ur;
        wave_sync();
        double uc = __builtin_huge_val();   // lane as row r
        double vr = __builtin_huge_val();   // lane as column q
        if (ok) {
            for (int q = 0; q < n; ++q) uc = __builtin_fmin(uc, sub_down((double)M[lane * n + q], sc.va[q]));
            for (int r = 0; r < n; ++r) vr = __builtin_fmin(vr, sub_down((double)M[r * n + lane], sc.vb[r]));
        }
        const double U = ok ? 0.5 * add_down(uc, (double)ur) : 0.0;    // lane as row
        const double V = ok ? 0.5 * add_down((double)vc, vr) : 0.0;    // lane as column
        wave_sync();
        sc.va[lane] = U;
        wave_sync();
        if (R != nullptr && ok) {
            for (int r = 0; r < n; ++r)
                R[r * n + lane] = to_float_down(sub_down(sub_down((double)M[r * n + lane], V), sc.va[r]));
        }
        if (duals != nullptr && ok) {
            duals[lane] = (T)uc;
            duals[n + lane] = vc;
            duals[2 * n + lane] = ur;
            duals[3 * n + lane] = (T)vr;
        }
        if (assign != nullptr && ok) assign[lane] = sig;
        const double su = S::sum_down(U);
        const double sv = S::sum_down(V);
        wave_sync();
        return add_down(su, sv);
    }
}

}  // namespace qap
