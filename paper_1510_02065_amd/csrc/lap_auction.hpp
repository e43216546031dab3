// Cost concentration by the auction algorithm: the assignment solver the
// paper's own GPU code uses (Section 6 of arXiv 1510.02065: one warp per
// problem, one thread per person; Bertsekas' auction with epsilon-scaling).
//
// Minimisation form.  Person r (a row) values object q (a column) at
// M_rq + p_q, p the object prices.  In a round every unassigned person finds
// its best object q1 (value w1) and second-best value w2 and bids the price
// p_q1 + (w2 - w1) + eps; each object goes to its highest bidder (ties to the
// lowest person), whose previous holder is unassigned again.  A phase ends
// when every person holds an object; eps then shrinks and the next phase
// starts from the current prices with every person unassigned.  The final
// assignment is within n eps of optimal.  Phases and rounds are bounded
// (AuctionEps, kAuctionMaxRounds), so a problem with non-finite entries ends.
//
// The dual handed to the residual does not depend on the assignment being
// complete or optimal: the row duals u_r = min_q (M_rq + p_q) and column duals
// v_q = -p_q are feasible for any prices, so the transferred value
// S = sum u + sum v is a lower bound on the assignment value (within n eps of
// it at the end of the last phase) and the residual M - u - v is >= 0.  The
// completion (lap_complete) raises each side to the minima left by the other,
// as for the canonical point.  Unlike the canonical dual this point depends
// on the solver's path, so the dual ascent it drives follows its own
// trajectory; its bound is valid but not the one the oracle computes.
//
// Layout: a segment of SEG >= n lanes per problem, lane l = person l for the
// bids and object l for the price and owner arrays in LDS (the problem's
// SlotScratch: u holds the prices, vb the bid keys, aux the owners, and the
// two short arrays together the winning person of each object's auction).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lap_slots.hpp"

namespace qap {

// Order-preserving map of a double to an unsigned 64-bit key (for the LDS
// maximum over bids).
__device__ __forceinline__ unsigned long long bid_key(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// eps of phase k is 2^-2 8^-k times the largest |M| of the problem: 13
// phases down to 2^-38 in FP64, 7 phases down to 2^-20 in FP32.
template <typename T>
struct AuctionEps {
    static constexpr int kPhases = sizeof(T) == 8 ? 13 : 7;
    static constexpr double kFirst = 0.25;
    static constexpr double kShrink = 0.125;
};

// Rounds of one phase after which the phase is abandoned (prices stay
// feasible duals whatever the assignment state).
constexpr int kAuctionMaxRounds = 1 << 14;

// Same contract as lap_concentrate_flat (one column per lane, n <= SEG):
// solve, write the residual (R, row stride ldr), duals [uc | vc | ur | vr],
// the assignment, and return S to every lane of the segment.
template <typename T, int SEG, bool DOWN>
__device__ __forceinline__ double lap_auction_flat(const SlotScratch<T, SEG, 1>& sc, int n, T* __restrict__ R,
                                                   long long ldr, T* __restrict__ duals,
                                                   int32_t* __restrict__ assign)
{
    using S = SegS<SEG>;
    const T* __restrict__ M = sc.M;
    const int ldm = sc.ld;   // row stride of M
    const int l = S::lane();
    const bool ok = l < n;
    double* __restrict__ price = sc.u;
    unsigned long long* __restrict__ key = reinterpret_cast<unsigned long long*>(sc.vb);
    int* __restrict__ owner = sc.aux;
    int* __restrict__ win = reinterpret_cast<int*>(sc.p);   // p and way: n ints together

    // Scale of the problem: the largest |M_rq|.
    double big = 0.0;
    if (ok)
        for (int q = 0; q < n; ++q) big = __builtin_fmax(big, __builtin_fabs((double)M[l * ldm + q]));
    big = -S::min(-big);
    if (ok) price[l] = 0.0;
    int my = -1;   // object held by person l
    wave_sync();

    // One phase per eps; a segment whose problem is all zeros (or empty)
    // needs no bidding and takes the identity below.
    double eps = big * AuctionEps<T>::kFirst;
    for (int phase = 0; phase < AuctionEps<T>::kPhases; ++phase, eps *= AuctionEps<T>::kShrink) {
        my = -1;
        if (ok) owner[l] = -1;
        wave_sync();
        for (int round = 0; round < kAuctionMaxRounds; ++round) {
            const bool bidding = ok && my < 0 && big > 0.0;
            if (ballot64(bidding) == 0) break;
            if (ok) {
                key[l] = 0ull;
                win[l] = SEG;
            }
            wave_sync();
            int q1 = 0;
            double newp = 0.0;
            unsigned long long mk = 0ull;
            if (bidding) {
                double w1 = __builtin_huge_val(), w2 = __builtin_huge_val();
                const T* __restrict__ Mr = M + l * ldm;
                for (int q = 0; q < n; ++q) {
                    const double val = (double)Mr[q] + price[q];
                    if (val < w1) {
                        w2 = w1;
                        w1 = val;
                        q1 = q;
                    } else if (val < w2) {
                        w2 = val;
                    }
                }
                if (n == 1) w2 = w1;
                newp = price[q1] + (w2 - w1) + eps;
                mk = bid_key(newp);
                atomicMax(&key[q1], mk);
            }
            wave_sync();
            if (bidding && key[q1] == mk) atomicMin(&win[q1], l);
            wave_sync();
            if (bidding && win[q1] == l) {
                owner[q1] = l;
                price[q1] = newp;
                my = q1;
            }
            wave_sync();
            if (ok && my >= 0 && owner[my] != l) my = -1;   // outbid
            wave_sync();
        }
    }
    // Persons left without an object (an abandoned phase, or an all-zero
    // problem) take the free objects in order, so the assignment is a
    // permutation.
    {
        const unsigned long long lanes = SegBits<SEG>::get(ok && my < 0);
        if (lanes != 0ull) {
            const unsigned long long freeo = SegBits<SEG>::get(ok && owner[ok ? l : 0] < 0);
            if (ok && my < 0) {
                const int rank = __builtin_popcountll(lanes & ((1ull << l) - 1ull));
                unsigned long long f = freeo;
                for (int k = 0; k < rank; ++k) f &= f - 1ull;
                my = f ? __builtin_ctzll(f) : 0;
            }
        }
    }
    wave_sync();
    // Feasible duals from the prices: u_r = min_q (M_rq + p_q), v_q = -p_q.
    T urow = (T)0, vcol = (T)0;
    if (ok) {
        double u = __builtin_huge_val();
        for (int q = 0; q < n; ++q) u = __builtin_fmin(u, (double)M[l * ldm + q] + price[q]);
        urow = (T)u;
        vcol = (T)(-price[l]);
    }
    wave_sync();
    const T vca[1] = {vcol};
    const T ura[1] = {urow};
    const int sga[1] = {my};
    return lap_complete<T, SEG, 1, DOWN>(sc, n, R, ldr, duals, assign, vca, ura, sga);
}

}  // namespace qap
