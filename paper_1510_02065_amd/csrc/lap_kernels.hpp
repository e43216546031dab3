// Cost-concentration kernels (Section 4.1 of arXiv 1510.02065).  Each wave
// works on 64/SEG assignment problems at once (one per SEG-lane segment), each
// staged in the wave's own LDS region; a workgroup holds WPB independent
// waves.  Problems of every instance of a handle are served by one launch per
// segment-size class.
#pragma once
#include "lap_auction.hpp"
#include "lap_slots.hpp"
#include "lap_wave.hpp"

namespace qap {

// Problems of a family, for the instances of one segment-size class:
// cls[0..Kc) are the instance ids and pre[] the prefix sums of their problem
// counts, so problem x belongs to instance cls[find_seg(pre, Kc, x)].
struct FamilyClass {
    const int* cls;
    const long long* pre;
    int Kc;
    long long total;
};

enum LapFamily : int { kFamD = 0, kFamC = 1 };

// How the D family is stored and enumerated (see pair_block).
enum DStorage : int {
    kAllBlocks = 0,    // every block stored (block-major); problem b is block b, parent c_b
    kHalfStore = 1,    // one block per complementary pair stored (pair-major);
                       // problem h is stored block h, parents c_beta and c_twin
    kHalfStoreTune = 2 // as kHalfStore, parent c_beta only (tuning runs)
};

// Copy an n x n block (row stride ld in global memory) into LDS (row stride
// ldm).  Each lane issues the loads of a whole chunk of rows before it writes
// any of them, so a wave waits for HBM once per chunk instead of once per row:
// the first kStageRows rows (all of them up to n = 24) in straight-line code,
// the rest kStageTail at a time.  Rows past the end re-read row n-1 and write
// it again (the same value to the same place), so no write is guarded.  Row
// offsets are 24-bit products: ld < 2^24 (at most N (N-1) (N-2) < 2^18 for
// N <= 64) and the offsets stay below 2^32 bytes.
constexpr int kStageRows = 24;
constexpr int kStageTail = 8;

template <typename T, int SEG, int K>
__device__ __forceinline__ void stage_block(T* __restrict__ M, int ldm, const T* __restrict__ blk, long long ld,
                                            int n, int lane)
{
    const unsigned ldb = (unsigned)ld * (unsigned)sizeof(T);   // row stride in bytes (< 2^24 * 8)
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int c = lane + k * SEG;
        if (c < n) {
            const char* __restrict__ col = reinterpret_cast<const char*>(blk + c);
            auto row_at = [&](int r) -> T {
                return *reinterpret_cast<const T*>(col + (size_t)(unsigned)__umul24((unsigned)r, ldb));
            };
            {
                T t[kStageRows];
#pragma unroll
                for (int u = 0; u < kStageRows; ++u) t[u] = row_at(min(u, n - 1));
#pragma unroll
                for (int u = 0; u < kStageRows; ++u) M[__umul24((unsigned)min(u, n - 1), (unsigned)ldm) + c] = t[u];
            }
            for (int r0 = kStageRows; r0 < n; r0 += kStageTail) {
                T t[kStageTail];
#pragma unroll
                for (int u = 0; u < kStageTail; ++u) t[u] = row_at(min(r0 + u, n - 1));
#pragma unroll
                for (int u = 0; u < kStageTail; ++u)
                    M[__umul24((unsigned)min(r0 + u, n - 1), (unsigned)ldm) + c] = t[u];
            }
        }
    }
}

// XCD-aware order of the assignment workgroups.  The hardware hands
// workgroup b to XCD b mod 8, and each XCD has its own L2; consecutive
// problems' block rows are adjacent in memory (they share the 128-byte lines
// at their ends), so each XCD takes one contiguous range of the workgroups'
// problems: workgroup b runs position xcd_major(b) of the problem order,
// ranges of q or q + 1 positions (q = grid / 8, the first grid % 8 XCDs
// taking one more).  A bijection of [0, grid).
__device__ __forceinline__ long long xcd_major(long long b, long long grid)
{
    const long long q = grid >> 3, r = grid & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Stage one problem per segment and solve it (the residual written over the
// block when blk is not null); S to every lane.  Called twice by the kernel
// below: with the size as a scalar (readfirstlane) when every problem of the
// wave has it, as in every wave of one instance's family, so that loop
// counts, clamps, bit masks and LDS offsets that depend only on n run on the
// scalar unit, and with the per-lane size otherwise (a wave across an
// instance boundary, or with segments past the last problem, whose n is 0).
// Both compute the same values.
template <typename T, int SEG, int K, bool AUC, bool DOWN>
__device__ __forceinline__ double stage_and_solve(unsigned char* smem, int seg, int lane, int nmax, int n, T* blk,
                                                  long long ld)
{
    const SlotScratch<T, SEG, K> sc(smem + seg * SlotLds<T, SEG, K>::bytes(nmax), n);
    stage_block<T, SEG, K>(sc.M, sc.ld, blk, ld, n, lane);
    wave_sync();
    static_assert(!AUC || K == 1, "the auction solver takes one column per lane");
    if constexpr (AUC)
        return lap_auction_flat<T, SEG, DOWN>(sc, n, blk, ld, nullptr, nullptr);
    else if constexpr (K == 1)
        return lap_concentrate_flat<T, SEG, DOWN>(sc, n, blk, ld, nullptr, nullptr);
    else if constexpr (SEG >= 16)
        return lap_concentrate_flatk<T, SEG, K, DOWN>(sc, n, blk, ld, nullptr, nullptr);
    else
        return lap_concentrate_slots<T, SEG, K, DOWN>(sc, n, blk, ld, nullptr, nullptr);
}

// D -> C (FAM kFamD: blocks D_beta of size N-2, parent c_beta) or C -> B
// (kFamC: blocks C_ij of size N-1, parent b_ij), K columns per lane, 64/SEG
// problems per wave, one wave per workgroup.  parent += S, the block is
// replaced by its residual, values[...] = S when values is not null (values
// are packed like the parents).  `mode` applies to the D family only.  AUC:
// the auction solver (one column per lane only).  Registers: with one
// column per lane the FP32 kernels are held to 72 VGPRs (seven waves per
// SIMD, about what their LDS allows at n = 23) and the FP64 ones of up to 32
// lanes to 80 (six waves: the LDS of the smaller problems of a batch allows
// more than the 99 VGPRs they would otherwise take); neither spills.
template <int PM, int SEG, int K, int FAM, bool AUC = false>
__global__ __launch_bounds__(64, K > 1 ? 1 : (PM != kPrecF64 ? 7 : (SEG <= 32 ? 6 : 1)))
void k_lap_family_s(StoreT<PM>* __restrict__ D, StoreT<PM>* __restrict__ C, StoreT<PM>* __restrict__ B,
                    const Inst* __restrict__ inst, FamilyClass fc, int nmax, double* __restrict__ values, int mode,
                    const int* __restrict__ act)
{
    using T = StoreT<PM>;
    constexpr bool DOWN = PM == kPrecF32Down;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int LPW = 64 / SEG;
    const int seg = threadIdx.x / SEG;
    const int lane = threadIdx.x & (SEG - 1);
    const long long x = xcd_major(blockIdx.x, gridDim.x) * LPW + seg;
    int kk = 0;
    if (x < fc.total) kk = find_seg(fc.pre, fc.Kc, x);
    const bool active = x < fc.total && act[fc.cls[kk]];
    int n = 0;
    T* blk = nullptr;
    long long ld = 0;   // row stride of the block in global memory
    long long pidx = 0, pidx2 = -1;
    if (active) {
        const Inst I = inst[fc.cls[kk]];
        const long long b = x - fc.pre[kk];
        if (FAM == kFamD) {
            n = I.N - 2;
            if (mode == kAllBlocks) {
                blk = D + I.offD + b * I.ldD;
                ld = n;
                pidx = I.offC + b;
            } else {
                long long beta, tb, base;
                pair_block(I.N, b, &beta, &tb, &base);
                blk = D + I.offD + base;
                ld = (long long)I.N * (I.N - 1) * n;
                pidx = I.offC + beta;
                if (mode == kHalfStore) pidx2 = I.offC + tb;
            }
        } else {
            n = I.N - 1;
            blk = C + I.offC + b * (long long)(I.N - 1) * (I.N - 1);
            ld = n;
            pidx = I.offB + b;
        }
    }
    const int nu = __builtin_amdgcn_readfirstlane(n);
    T* const bw = active ? blk : nullptr;
    const double S = ballot64(n != nu) == 0
                         ? stage_and_solve<T, SEG, K, AUC, DOWN>(smem, seg, lane, nmax, nu, bw, ld)
                         : stage_and_solve<T, SEG, K, AUC, DOWN>(smem, seg, lane, nmax, n, bw, ld);
    if (active && lane == 0) {
        T* parent = (FAM == kFamD) ? C : B;
        parent[pidx] = store_add<PM>(parent[pidx], S);
        if (pidx2 >= 0) parent[pidx2] = store_add<PM>(parent[pidx2], S);
        if (values) {
            values[pidx] = S;
            if (pidx2 >= 0) values[pidx2] = S;
        }
    }
}

// B -> LB' and LB += LB' (steps 7-8), one problem of size N per instance of
// the class, K columns per lane.  lb[2k] = LB, lb[2k+1] = LB' (FP64; in FP32
// certified mode the bound accumulates rounding toward -inf).  The instance's
// trace gets (LB, LB') at position counter[k]++ when below trace_cap, and
// sigma (nullable, packed like B) the assignment of the B problem, a
// permutation of the instance.  Stop rule of Algorithm 1, with stop[0] = K and
// stop[1] = UB (UB <= 0: none): the instance's act flag is cleared once
// LB >= UB or LB' / UB < K.
template <int PM, int SEG, int K, bool AUC = false>
__global__ __launch_bounds__(64) void k_lap_B_s(StoreT<PM>* __restrict__ B, const Inst* __restrict__ inst,
                                                FamilyClass fc, int nmax, double* __restrict__ lb,
                                                double* __restrict__ trace, long long* __restrict__ counter,
                                                long long trace_cap, double* __restrict__ values,
                                                int32_t* __restrict__ sigma, int* __restrict__ act,
                                                const double* __restrict__ stop)
{
    using T = StoreT<PM>;
    constexpr bool DOWN = PM == kPrecF32Down;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int LPW = 64 / SEG;
    const int seg = threadIdx.x / SEG;
    const int lane = threadIdx.x & (SEG - 1);
    const long long x = (long long)blockIdx.x * LPW + seg;
    const int k = x < fc.total ? fc.cls[x] : 0;
    const bool active = x < fc.total && act[k];
    const Inst I = inst[k];
    const int n = active ? I.N : 0;
    T* blk = B + I.offB;
    const SlotScratch<T, SEG, K> sc(smem + seg * SlotLds<T, SEG, K>::bytes(nmax), n);
    stage_block<T, SEG, K>(sc.M, sc.ld, blk, n, n, lane);
    wave_sync();
    int32_t* sg = (active && sigma) ? sigma + I.offB : nullptr;
    double S;
    static_assert(!AUC || K == 1, "the auction solver takes one column per lane");
    if constexpr (AUC)
        S = lap_auction_flat<T, SEG, DOWN>(sc, n, active ? blk : nullptr, n, nullptr, sg);
    else if constexpr (K == 1)
        S = lap_concentrate_flat<T, SEG, DOWN>(sc, n, active ? blk : nullptr, n, nullptr, sg);
    else if constexpr (SEG >= 16)
        S = lap_concentrate_flatk<T, SEG, K, DOWN>(sc, n, active ? blk : nullptr, n, nullptr, sg);
    else
        S = lap_concentrate_slots<T, SEG, K, DOWN>(sc, n, active ? blk : nullptr, n, nullptr, sg);
    if (active && lane == 0) {
        const double L = DOWN ? add_down(lb[2 * k], S) : lb[2 * k] + S;
        lb[2 * k] = L;
        lb[2 * k + 1] = S;
        if (values) values[k] = S;
        if (counter) {
            const long long t = counter[k];
            if (trace && t < trace_cap) {
                trace[(k * trace_cap + t) * 2] = L;
                trace[(k * trace_cap + t) * 2 + 1] = S;
            }
            counter[k] = t + 1;
        }
        const double Kp = stop[0], UB = stop[1];
        if (UB > 0.0 && (L >= UB || (Kp > 0.0 && S < Kp * UB))) act[k] = 0;
    }
}

// Generic batch (qap_lap_solve): launch slot s < count solves problem
// b = idx[s] (b = s when idx is null); count = *dcount when dcount is not
// null, else `count`.  Problem b has size n[b] (<= SEG, else its value is NaN
// and nothing else is written), matrix at cost + mat_off[b], vectors at
// vec_off[b] (vec_off may be null when duals and assign are).  AUC: the
// auction solver (lap_auction_flat) instead of the canonical dual.
template <int PM, int SEG, bool AUC>
__global__ __launch_bounds__(64) void k_lap_batch(int count, const int* __restrict__ dcount,
                                                  const int32_t* __restrict__ idx, const int32_t* __restrict__ nv,
                                                  const int64_t* __restrict__ mat_off,
                                                  const int64_t* __restrict__ vec_off,
                                                  StoreT<PM>* __restrict__ cost, double* __restrict__ value,
                                                  StoreT<PM>* __restrict__ duals, int32_t* __restrict__ assign,
                                                  int write_residual)
{
    using T = StoreT<PM>;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int LPW = 64 / SEG;
    const int seg = threadIdx.x / SEG;
    const int lane = threadIdx.x & (SEG - 1);
    const int cnt = dcount ? *dcount : count;
    const int64_t s = (int64_t)blockIdx.x * LPW + seg;
    const bool in = s < cnt;
    const int64_t b = in ? (idx ? (int64_t)idx[s] : s) : 0;
    int n = in ? nv[b] : 0;
    const bool bad = n < 0 || n > SEG;
    if (bad) n = 0;
    T* mat = (in && !bad) ? cost + mat_off[b] : nullptr;
    const int64_t vo = (in && !bad && vec_off) ? vec_off[b] : 0;
    T* const Rw = (write_residual && n > 0) ? mat : nullptr;
    T* const dw = (duals && n > 0) ? duals + 4 * vo : nullptr;
    int32_t* const aw = (assign && n > 0) ? assign + vo : nullptr;
    // The size as a scalar when every problem of the wave has it, as in
    // k_lap_family_s.
    auto solve = [&](int nn) __attribute__((always_inline)) -> double {
        const SlotScratch<T, SEG, 1> sc(smem + seg * SlotLds<T, SEG, 1>::bytes(SEG), nn);
        stage_block<T, SEG, 1>(sc.M, sc.ld, mat, nn, nn, lane);
        wave_sync();
        if constexpr (AUC)
            return lap_auction_flat<T, SEG, PM == kPrecF32Down>(sc, nn, Rw, nn, dw, aw);
        else
            return lap_concentrate_flat<T, SEG, PM == kPrecF32Down>(sc, nn, Rw, nn, dw, aw);
    };
    const int nu = __builtin_amdgcn_readfirstlane(n);
    const double S = ballot64(n != nu) == 0 ? solve(nu) : solve(n);
    // A quiet NaN written by bit pattern marks a problem that was not solved.
    if (in && lane == 0) value[b] = bad ? __longlong_as_double(0x7ff8000000000000ll) : S;
}

}  // namespace qap
