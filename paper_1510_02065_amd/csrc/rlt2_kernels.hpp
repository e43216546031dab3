// Element-wise kernels of the RLT2 dual ascent on gfx950: initial dual,
// cost spreading and the transfers between complementary coefficients
// (Sections 3, 4.2 and 4.3 of arXiv 1510.02065), plus the FP64 certification
// cascade.
//
// Layouts (compact, block-major; every block holds its rows and columns in
// ascending original index with the excluded indices skipped):
//   B  [i*N + j]
//   C  block (i,j) of (N-1)^2 entries at (i*N+j)*(N-1)^2; entry (k', n').
//      beta(ijkn) = (i*N+j)*(N-1)^2 + k'*(N-1) + n', k' = k-[k>i], n' = n-[n>j].
//   D  block D_ijkn is block number beta(ijkn), at beta*ldD (ldD >= (N-2)^2,
//      padded so that every block starts on a 128-byte boundary); entry
//      (p'', q''), p'' = p-[p>min(i,k)]-[p>max(i,k)], q'' likewise with j, n.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace qap {

__device__ __forceinline__ int skip1(int r, int a) { return r + (r >= a); }
// r-th index (0-based, ascending) that is neither lo nor hi (lo < hi).
__device__ __forceinline__ int skip2(int r, int lo, int hi) {
    r += (r >= lo);
    r += (r >= hi);
    return r;
}
__device__ __forceinline__ int drop1(int x, int a) { return x - (x > a); }
__device__ __forceinline__ int drop2(int x, int a, int b) { return x - (x > a) - (x > b); }

// ---- arithmetic of the three precisions -------------------------------------
// FP64 mode: plain IEEE round-to-nearest; the element-wise steps perform
// exactly the operations of the algorithm in the same order as a plain
// sequential reference, and so match it bit for bit.
//
// FP32 nearest mode: reduced costs are stored as floats; every value written
// into the state is computed in FP64 with the FP64 mode's operations (the
// six-way mean multiplying by 1/6 instead of dividing by 6) and rounded to
// nearest once, so the FP32 state follows the FP64 trajectory without a
// systematic bias.
//
// FP32 certified mode: reduced costs are stored as floats, and every value
// written into the state (B, C, D, LB) is computed in FP64 and rounded
// toward -inf exactly once.  Rounding down can only lower what the state
// represents for a permutation, so the represented objective never exceeds
// the true one and LB stays a valid lower bound.  The directed FP64 steps
// are built from round-to-nearest operations with their exact errors
// (TwoSum for sums, the FMA residual for products and quotients), so no
// hardware rounding mode is changed.

// The next representable value below x (x finite).
__device__ __forceinline__ double next_down(double x) {
    if (x == 0.0) return -__longlong_as_double(1ll);
    const long long b = __double_as_longlong(x);
    return __longlong_as_double(x > 0.0 ? b - 1 : b + 1);
}
__device__ __forceinline__ float next_down(float x) {
    if (x == 0.0f) return -__int_as_float(1);
    const int b = __float_as_int(x);
    return __int_as_float(x > 0.0f ? b - 1 : b + 1);
}
// a + b rounded toward -inf.
__device__ __forceinline__ double add_down(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    const double err = (a - (s - bb)) + (b - bb);
    return err < 0.0 ? next_down(s) : s;
}
__device__ __forceinline__ double sub_down(double a, double b) { return add_down(a, -b); }
// a * b rounded toward -inf.
__device__ __forceinline__ double mul_down(double a, double b) {
    const double p = a * b;
    const double err = __builtin_fma(a, b, -p);
    return err < 0.0 ? next_down(p) : p;
}
// a / m rounded toward -inf (m > 0): q*m - a is exact in an FMA.
__device__ __forceinline__ double div_down(double a, double m) {
    const double q = a / m;
    const double r = __builtin_fma(q, m, -a);
    return r > 0.0 ? next_down(q) : q;
}
// Largest float <= x.
__device__ __forceinline__ float to_float_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = next_down(f);
    return f;
}
// Largest float <= x, for x >= 0: a nearest float above x is then positive,
// so the float below it is its bit pattern minus one.
__device__ __forceinline__ float to_float_down_nonneg(double x) {
    const float f = (float)x;
    return (double)f > x ? __int_as_float(__float_as_int(f) - 1) : f;
}
__device__ __forceinline__ float mul_down_to_float(double a, double b) {
    const double p = a * b;
    const double err = __builtin_fma(a, b, -p);
    float f = (float)p;
    if ((double)f > p || ((double)f == p && err < 0.0)) f = next_down(f);
    return f;
}
__device__ __forceinline__ float add_down_to_float(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    const double err = (a - (s - bb)) + (b - bb);
    float f = (float)s;
    if ((double)f > s || ((double)f == s && err < 0.0)) f = next_down(f);
    return f;
}

// Mean of the six member sums (d_m + x_m), m = 0..5, of one six-way group,
// rounded toward -inf, for the FP32 certified mode (the terms are the stored
// members and their spread shares, as floats).  When every term is >= 0 the
// round-to-nearest FP64 sum (m_0 + ... + m_5, each m = d + x) is within
// (1 + 2^-53)^6 - 1 < 7 * 2^-53 of the exact sum, relatively; multiplying by
// 1/6 (two more roundings) and by 1 - 2^-48 therefore gives a value below the
// exact mean, and its largest float below is written.  That is at most one
// FP32 step below the directed result, for a fraction of the work of
// rounding every step toward -inf, which is what happens when a term is
// negative (a state loaded by the caller may hold such entries).
// The path for terms of either sign is a call, kept out of line so that the
// sweeps' registers are sized for the common path.
__device__ __attribute__((noinline)) float mean6_down_signed(float d0, float x0, float d1, float x1, float d2,
                                                            float x2, float d3, float x3, float d4, float x4,
                                                            float d5, float x5);
__device__ __forceinline__ float mean6_down(float d0, float x0, float d1, float x1, float d2, float x2, float d3,
                                            float x3, float d4, float x4, float d5, float x5)
{
    const float lo = fminf(fminf(fminf(fminf(d0, x0), fminf(d1, x1)), fminf(fminf(d2, x2), fminf(d3, x3))),
                           fminf(fminf(d4, x4), fminf(d5, x5)));
    if (lo >= 0.0f) {
        double sum = (double)d0 + (double)x0;
        sum += (double)d1 + (double)x1;
        sum += (double)d2 + (double)x2;
        sum += (double)d3 + (double)x3;
        sum += (double)d4 + (double)x4;
        sum += (double)d5 + (double)x5;
        return to_float_down_nonneg((sum * (1.0 / 6.0)) * (1.0 - 0x1p-48));
    }
    return mean6_down_signed(d0, x0, d1, x1, d2, x2, d3, x3, d4, x4, d5, x5);
}
__device__ __attribute__((noinline)) float mean6_down_signed(float d0, float x0, float d1, float x1, float d2,
                                                            float x2, float d3, float x3, float d4, float x4,
                                                            float d5, float x5)
{
    double sum = add_down((double)d0, (double)x0);
    sum = add_down(sum, (double)d1);
    sum = add_down(sum, (double)x1);
    sum = add_down(sum, (double)d2);
    sum = add_down(sum, (double)x2);
    sum = add_down(sum, (double)d3);
    sum = add_down(sum, (double)x3);
    sum = add_down(sum, (double)d4);
    sum = add_down(sum, (double)x4);
    sum = add_down(sum, (double)d5);
    sum = add_down(sum, (double)x5);
    return to_float_down(div_down(sum, 6.0));
}

// Precision modes (the values of qap_precision).  kPrecF64: FP64 state,
// round-to-nearest.  kPrecF32Down: FP32 state, every value written rounded
// toward -inf once (the represented objective can only fall, a proof of
// validity).  kPrecF32Near: FP32 state, every value computed in FP64 and
// rounded to nearest once (no systematic drift; validity rests on the FP64
// certification over the stored state).
enum PrecMode : int { kPrecF64 = 0, kPrecF32Down = 1, kPrecF32Near = 2 };
template <int PM>
using StoreT = typename std::conditional<PM == kPrecF64, double, float>::type;

// An FP64 value as written into the state of mode PM.
template <int PM>
__device__ __forceinline__ StoreT<PM> store_val(double x) {
    if constexpr (PM == kPrecF64)
        return x;
    else if constexpr (PM == kPrecF32Down)
        return to_float_down(x);
    else
        return (float)x;
}
// parent + S (S in FP64) as written into the state of mode PM.
template <int PM>
__device__ __forceinline__ StoreT<PM> store_add(StoreT<PM> parent, double S) {
    if constexpr (PM == kPrecF64)
        return parent + S;
    else if constexpr (PM == kPrecF32Down)
        return to_float_down(add_down((double)parent, S));
    else
        return (float)((double)parent + S);
}

// Block number of D_{(a,la),(b,lb)} (= position of c_{a la b lb} in C).
__device__ __forceinline__ int64_t beta_of(int N, int a, int la, int b, int lb) {
    const int n1 = N - 1;
    return ((int64_t)(a * N + la) * n1 + drop1(b, a)) * n1 + drop1(lb, la);
}
// Complementary blocks (Section 6): D_{(a,la),(b,lb)} and D_{(b,lb),(a,la)}
// cover the same rows and columns, and entry (c,lc) of each belongs to the
// same six-way group of equation (11).  The six-way transfer leaves every
// member of a group with the same value and a concentration leaves both blocks
// with the same residual, so from D = 0 on the two blocks are always equal:
// the handle can store one copy, the block with a < b.
//
// Pair-major layout of those stored blocks.  Row c of block (a,la,b,lb)
// (facility c not in {a, b}) holds the entries whose six-way groups belong to
// facility triple {a, b, c}, so the layout keeps, for each facility pair
// a < b and each row c, the rows of all N (N-1) location pairs (la, lb)
// together:
//   offset = ((P(a,b) (N-2) + c') N(N-1) + L(la,lb)) (N-2) + lc',
// P(a,b) the lexicographic index of the pair, c' = c - [c > a] - [c > b],
// L(la,lb) = la (N-1) + lb - [lb > la], lc' the compact column.  The steps
// 1-3 pass over triple {x < y < z} then reads three contiguous runs of
// N (N-1) (N-2) entries, and an assignment problem reads its block as N-2
// rows, N (N-1) (N-2) entries apart.

__host__ __device__ __forceinline__ long long pair_index(int N, int a, int b)   // a < b
{
    return (long long)a * (2 * N - a - 1) / 2 + (b - a - 1);
}

// Offset of row c' (compact) of stored block (a, la, b, lb), a < b.
__host__ __device__ __forceinline__ long long pair_row(int N, int a, int la, int b, int lb, int cq)
{
    const long long NL = (long long)N * (N - 1);
    const int n2 = N - 2;
    return ((pair_index(N, a, b) * n2 + cq) * NL + (long long)la * (N - 1) + (lb - (lb > la))) * n2;
}

// Stored block number h in [0, N^2 (N-1)^2 / 2) = P(a,b) N(N-1) + L(la,lb):
// *beta gets the block number (position of its c in C), *twin that of its
// complement and *base the offset of its first row (rows are
// N (N-1) (N-2) apart).
// The quotients are taken in FP32 and corrected once: h < N^2 (N-1)^2 / 2 <
// 2^23 for N <= 64 is exact in FP32 and the computed quotient is within
// 2^-22 relative (less than 1/2) of the true one.  Facility a of pair index
// P is the largest a with S(a) = a (2N - a - 1) / 2 <= P, from the root of
// that quadratic, corrected the same way.
__host__ __device__ __forceinline__ void pair_block(int N, long long h, long long* beta, long long* twin,
                                                    long long* base)
{
    const int n1 = N - 1;
    const int NL = N * n1;
    const int hh = (int)h;
    int P = (int)((float)hh * (1.0f / (float)NL));
    int L = hh - P * NL;
    if (L < 0) {
        --P;
        L += NL;
    } else if (L >= NL) {
        ++P;
        L -= NL;
    }
    // 32-bit products up to the last multiplication (block numbers are below
    // N^2 (N-1)^2 < 2^24); the first-row offset needs 64 bits.
    *base = (long long)(((unsigned long long)(unsigned)(P * (N - 2)) * (unsigned)NL + (unsigned)L) * (unsigned)(N - 2));
    const float tw = (float)(2 * N - 1);
    int a = (int)((tw - sqrtf(tw * tw - 8.0f * (float)P)) * 0.5f);
    if (a * (2 * N - a - 1) / 2 > P) --a;
    else if ((a + 1) * (2 * N - a - 2) / 2 <= P) ++a;
    const int b = a + 1 + (P - a * (2 * N - a - 1) / 2);
    int la = (int)((float)L * (1.0f / (float)n1));
    int lq = L - la * n1;
    if (lq < 0) {
        --la;
        lq += n1;
    } else if (lq >= n1) {
        ++la;
        lq -= n1;
    }
    const int lb = lq + (lq >= la);
    *beta = ((a * N + la) * n1 + (b - 1)) * n1 + lq;
    *twin = ((b * N + lb) * n1 + a) * n1 + (la - (la > lb));
}

// Offset of d_{(a,la),(b,lb),(c,lc)} inside block beta_of(a,la,b,lb).
__device__ __forceinline__ int entry_of(int N, int a, int la, int b, int lb, int c, int lc) {
    return drop2(c, a, b) * (N - 2) + drop2(lc, la, lb);
}

// ---- instances -----------------------------------------------------------------
// A handle holds K independent instances (a single QAP, or the nodes of a
// branch-and-bound batch).  Their B, C and D arrays are packed one after the
// other; every kernel below covers all instances in one launch and finds its
// instance by binary search in a prefix array.  The iteration kernels also take
// act[], one flag per instance: 1 while its dual ascent runs, 0 once the stop
// rule of Algorithm 1 has ended it, after which they leave its state as it is.
struct Inst {
    int N;
    int ntri;          // N(N-1)(N-2)/6 facility triples
    int wpt;           // sweep workgroups per facility triple
    int pad_;
    long long offB;    // first entry of the instance in the packed B array
    long long offC;    // first entry in the packed C (and CC) arrays
    long long offD;    // first entry in the packed D array
    long long ldD;     // block stride of D (>= (N-2)^2, 128-byte multiple)
    long long wg0;     // first sweep workgroup (a multiple of 8)
    long long tri0;    // first int of the instance's facility-triple table
};

// Largest k in [0, K) with pre[k] <= x (pre ascending, pre[0] = 0).
__device__ __forceinline__ int find_seg(const long long* __restrict__ pre, int K, long long x) {
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Initial dual of one instance (the lines of Algorithm 1 before its loop):
//   b_ij = f_ii d_jj (+ B0_ij), c_ijkn = f_ik d_jn.
template <int PM>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ F, const double* __restrict__ Dm,
                                              const double* __restrict__ B0, StoreT<PM>* __restrict__ B,
                                              StoreT<PM>* __restrict__ C, int N)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n1 = N - 1;
    const int64_t nC = (int64_t)N * N * n1 * n1;
    if (x < (int64_t)N * N) {
        const int i = (int)(x / N), j = (int)(x % N);
        if constexpr (PM == kPrecF32Down) {
            const double b = mul_down(F[i * N + i], Dm[j * N + j]);
            B[x] = add_down_to_float(b, B0 ? B0[x] : 0.0);
        } else {
            double b = F[i * N + i] * Dm[j * N + j];
            if (B0) b = b + B0[x];
            B[x] = (StoreT<PM>)b;
        }
    }
    if (x < nC) {
        const int ij = (int)(x / (n1 * n1));
        const int rem = (int)(x % (n1 * n1));
        const int i = ij / N, j = ij % N;
        const int k = skip1(rem / n1, i), n = skip1(rem % n1, j);
        if constexpr (PM == kPrecF32Down)
            C[x] = mul_down_to_float(F[i * N + k], Dm[j * N + n]);
        else
            C[x] = (StoreT<PM>)(F[i * N + k] * Dm[j * N + n]);
    }
}


// Steps 1-2 precomputation, one thread per C entry of every instance: the
// amount each entry of block D_beta receives,
//   CC_beta = (c_beta + b_ij / (N-1)) / (N-2),
// after which c is cleared (B is cleared by the sweep, which does not read it).
template <int PM>
__global__ __launch_bounds__(256) void k_spread_prep(StoreT<PM>* __restrict__ C, const StoreT<PM>* __restrict__ B,
                                                     StoreT<PM>* __restrict__ CC, const Inst* __restrict__ inst,
                                                     const long long* __restrict__ preC, int K,
                                                     long long totalC, const int* __restrict__ act)
{
    using T = StoreT<PM>;
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= totalC) return;
    const int kk = find_seg(preC, K, x);
    if (!act[kk]) return;
    const Inst I = inst[kk];
    const int N = I.N, n1 = N - 1;
    const int ij = (int)((x - I.offC) / (n1 * n1));
    const T bij = B[I.offB + ij];
    if constexpr (PM == kPrecF32Down) {
        const double c = add_down((double)C[x], div_down((double)bij, (double)(N - 1)));
        CC[x] = to_float_down(div_down(c, (double)(N - 2)));
    } else {
        const double share_b = (double)bij / (double)(N - 1);
        const double c = (double)C[x] + share_b;
        CC[x] = (T)(c / (double)(N - 2));
    }
    C[x] = (T)0;
}

// Step 1 alone (the level-1 dual ascent, which has no D): c += b_ij / (N-1)
// over every C entry of the active instances.  B is cleared by k_clear_B.
template <int PM>
__global__ __launch_bounds__(256) void k_spread_B(StoreT<PM>* __restrict__ C, const StoreT<PM>* __restrict__ B,
                                                  const Inst* __restrict__ inst, const long long* __restrict__ preC,
                                                  int K, long long totalC, const int* __restrict__ act)
{
    using T = StoreT<PM>;
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= totalC) return;
    const int kk = find_seg(preC, K, x);
    if (!act[kk]) return;
    const Inst I = inst[kk];
    const int N = I.N, n1 = N - 1;
    const int ij = (int)((x - I.offC) / (n1 * n1));
    const T bij = B[I.offB + ij];
    if constexpr (PM == kPrecF32Down)
        C[x] = to_float_down(add_down((double)C[x], div_down((double)bij, (double)(N - 1))));
    else
        C[x] = (T)((double)C[x] + (double)bij / (double)(N - 1));
}

// b = 0 over the active instances (after step 1 of the level-1 ascent).
template <int PM>
__global__ __launch_bounds__(256) void k_clear_B(StoreT<PM>* __restrict__ B, const long long* __restrict__ preB,
                                                 int K, long long totalB, const int* __restrict__ act)
{
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= totalB) return;
    if (act[find_seg(preB, K, x)]) B[x] = (StoreT<PM>)0;
}

// The sweep kernels clear instance I's B (N^2 entries) from the workgroup
// that takes the instance's first facility triple.
template <typename T>
__device__ __forceinline__ void clear_inst_B(T* __restrict__ B, const Inst& I, int tid, int nthreads)
{
    for (int e = tid; e < I.N * I.N; e += nthreads) B[I.offB + e] = (T)0;
}

// Steps 1-3 on D: every entry gets its block's spread share, then each group
// of six complementary coefficients (equation (11)) is replaced by its mean.
// One thread per group.  A group is an unordered triple of (facility,
// location) pairs; it is enumerated as a facility triple i < k < p (from the
// instance's triple table) times an ordered location triple (j, n, q) of
// distinct locations, with q varying fastest so that the members (P1 P2 P3)
// and (P2 P1 P3) are read and written contiguously.  With P1=(i,j), P2=(k,n),
// P3=(p,q) the six members are summed in lexicographic order of the
// permutation of (P1, P2, P3), so the result is the same bits on every run.
//
// XCD-aware schedule: the hardware hands workgroup b to XCD b mod 8, and each
// XCD has its own L2.  Within an instance (whose first workgroup is a
// multiple of 8) all wpt workgroups of facility triple t get ids congruent to
// t mod 8 and consecutive among that XCD's ids, so one XCD works through a
// triple's six sub-arrays (6 N(N-1)(N-2) entries) together and the partially
// used cache lines of the four strided members meet in its L2.
// The first totalB threads of the grid also clear B.  Used when every block
// is stored; see k_sweep_cube for one block per complementary pair.
template <int PM>
__global__ __launch_bounds__(256) void k_sweep(StoreT<PM>* __restrict__ Dd, const StoreT<PM>* __restrict__ CC,
                                               StoreT<PM>* __restrict__ B, const int* __restrict__ tri,
                                               const Inst* __restrict__ inst,
                                               const long long* __restrict__ preWG, int K,
                                               const int* __restrict__ act)
{
    using T = StoreT<PM>;
    const int kk = find_seg(preWG, K, (long long)blockIdx.x);
    if (!act[kk]) return;   // whole workgroup
    const Inst I = inst[kk];
    const int lb = (int)((long long)blockIdx.x - I.wg0);
    if (lb == 0) clear_inst_B(B, I, threadIdx.x, 256);
    const int xcd = lb & 7;
    const int local = lb >> 3;
    const int t = (local / I.wpt) * 8 + xcd;
    const int w = local % I.wpt;
    if (t >= I.ntri) return;
    const int N = I.N, n1 = N - 1, n2 = N - 2;
    const int L = N * n1 * n2;
    const int loc = w * 256 + (int)threadIdx.x;
    if (loc >= L) return;
    const int qq = loc % n2;
    const int rest = loc / n2;
    const int j = rest / n1;
    const int n = skip1(rest % n1, j);
    const int q = skip2(qq, min(j, n), max(j, n));
    const int* tr = tri + I.tri0 + 3 * t;
    const int i = tr[0], k = tr[1], p = tr[2];
    T* __restrict__ Dk = Dd + I.offD;
    const T* __restrict__ CCk = CC + I.offC;
    const long long ldD = I.ldD;

    const int64_t b0 = beta_of(N, i, j, k, n), b1 = beta_of(N, i, j, p, q);
    const int64_t b2 = beta_of(N, k, n, i, j), b3 = beta_of(N, k, n, p, q);
    const int64_t b4 = beta_of(N, p, q, i, j), b5 = beta_of(N, p, q, k, n);
    const int64_t a0 = b0 * ldD + entry_of(N, i, j, k, n, p, q);
    const int64_t a1 = b1 * ldD + entry_of(N, i, j, p, q, k, n);
    const int64_t a2 = b2 * ldD + entry_of(N, k, n, i, j, p, q);
    const int64_t a3 = b3 * ldD + entry_of(N, k, n, p, q, i, j);
    const int64_t a4 = b4 * ldD + entry_of(N, p, q, i, j, k, n);
    const int64_t a5 = b5 * ldD + entry_of(N, p, q, k, n, i, j);

    T mean;
    if constexpr (PM != kPrecF32Down) {
        const double m0 = (double)Dk[a0] + (double)CCk[b0];
        const double m1 = (double)Dk[a1] + (double)CCk[b1];
        const double m2 = (double)Dk[a2] + (double)CCk[b2];
        const double m3 = (double)Dk[a3] + (double)CCk[b3];
        const double m4 = (double)Dk[a4] + (double)CCk[b4];
        const double m5 = (double)Dk[a5] + (double)CCk[b5];
        double s = m0;
        s += m1;
        s += m2;
        s += m3;
        s += m4;
        s += m5;
        // FP64: IEEE division (the oracle's operation, bit for bit); FP32
        // nearest: the FP64 sum times 1/6, rounded to float once (the
        // division's correctly rounded FP64 quotient would only matter for
        // the rare sum within one FP64 ulp of a float rounding boundary).
        if constexpr (PM == kPrecF64)
            mean = (T)(s / 6.0);
        else
            mean = (T)(s * (1.0 / 6.0));
    } else {
        mean = mean6_down(Dk[a0], CCk[b0], Dk[a1], CCk[b1], Dk[a2], CCk[b2], Dk[a3], CCk[b3], Dk[a4], CCk[b4],
                          Dk[a5], CCk[b5]);
    }
    Dk[a0] = mean;
    Dk[a1] = mean;
    Dk[a2] = mean;
    Dk[a3] = mean;
    Dk[a4] = mean;
    Dk[a5] = mean;
}

// Steps 1-3 with one stored block per complementary pair (pair_row).  As
// i < k < p, members (P1 P2 P3) and (P2 P1 P3) share one stored entry A,
// (P1 P3 P2) and (P3 P1 P2) share B, and (P2 P3 P1) and (P3 P2 P1) share C;
// each member still gets its own block's spread share, in k_sweep's order,
// so the sum has the same bits as with every block stored.
//
// Workgroups: kSweepParts per facility triple, on one XCD (ids congruent to
// the triple mod 8, as in k_sweep, so lines shared between them meet in that
// XCD's L2).  A workgroup first stages the six N x N tables of spread shares
// of its triple in LDS (X[m][a][b] = CC of block (f1, a, f2, b) for the six
// ordered facility pairs), so the groups read them from LDS instead of
// making scattered L2 requests.  Each wave then takes 4 x 4 x 4 cubes of
// location triples (j, n, q), two at a time:
//   A = D_{(i,j),(k,n)}[p][q]  (contiguous over q),
//   B = D_{(i,j),(p,q)}[k][n]  (contiguous over n),
//   C = D_{(k,n),(p,q)}[i][j]  (contiguous over j),
// each in the triple's own run of the pair-major layout, so each member's 64
// lanes fall on 16 runs of 4 consecutive entries.  Groups with a repeated
// location and cube cells past N are masked off.  STAGE = false (tables too
// large for LDS, N > 58 in FP64) reads the spread shares from global memory.
constexpr int kSweepParts = 8;

template <int PM, typename T = StoreT<PM>>
__device__ __forceinline__ T six_way_mean(T A0, T B0, T C0, T x0, T x1, T x2, T x3, T x4, T x5)
{
    if constexpr (PM != kPrecF32Down) {
        const double m0 = (double)A0 + (double)x0;
        const double m1 = (double)B0 + (double)x1;
        const double m2 = (double)A0 + (double)x2;
        const double m3 = (double)C0 + (double)x3;
        const double m4 = (double)B0 + (double)x4;
        const double m5 = (double)C0 + (double)x5;
        double sum = m0;
        sum += m1;
        sum += m2;
        sum += m3;
        sum += m4;
        sum += m5;
        if constexpr (PM == kPrecF64)
            return (T)(sum / 6.0);   // the oracle's operation, bit for bit
        else
            return (T)(sum * (1.0 / 6.0));   // rounded to float once (see k_sweep)
    } else {
        return mean6_down(A0, x0, B0, x1, A0, x2, C0, x3, B0, x4, C0, x5);
    }
}

template <int PM, bool STAGE>
__global__ __launch_bounds__(256) void k_sweep_cube(StoreT<PM>* __restrict__ Dd, const StoreT<PM>* __restrict__ CC,
                                                    StoreT<PM>* __restrict__ B, const int* __restrict__ tri,
                                                    const Inst* __restrict__ inst,
                                                    const long long* __restrict__ preWG, int K, int Nmax,
                                                    const int* __restrict__ act)
{
    using T = StoreT<PM>;
    extern __shared__ __align__(16) unsigned char smem[];
    T* __restrict__ X = reinterpret_cast<T*>(smem);   // [6][Nmax][Nmax]
    const int kk = find_seg(preWG, K, (long long)blockIdx.x);
    if (!act[kk]) return;   // whole workgroup
    const Inst I = inst[kk];
    const int lbk = (int)((long long)blockIdx.x - I.wg0);
    if (lbk == 0) clear_inst_B(B, I, threadIdx.x, 256);
    const int xcd = lbk & 7;
    const int local = lbk >> 3;
    const int t = (local / kSweepParts) * 8 + xcd;
    if (t >= I.ntri) return;   // whole workgroup
    const int part = local % kSweepParts;
    const int N = I.N, n1 = N - 1, n2 = N - 2;
    const int* tr = tri + I.tri0 + 3 * t;
    const int i = tr[0], k = tr[1], p = tr[2];
    T* __restrict__ Dk = Dd + I.offD;
    const T* __restrict__ CCk = CC + I.offC;

    // Spread shares of the triple: X[m][a][b] = CC of block (f1_m, a, f2_m, b),
    // (f1, f2) = (i,k), (i,p), (k,i), (k,p), (p,i), (p,k).
    const int NN = Nmax * Nmax;
    if constexpr (STAGE) {
        for (int x = threadIdx.x; x < 6 * N * N; x += 256) {
            const int m = x / (N * N), r = x - m * N * N;
            const int a = r / N, b = r - a * N;
            if (a == b) continue;
            const int f1 = m < 2 ? i : m < 4 ? k : p;
            const int f2 = (m == 0 || m == 5) ? k : (m == 1 || m == 3) ? p : i;
            X[m * NN + a * Nmax + b] = CCk[beta_of(N, f1, a, f2, b)];
        }
        __syncthreads();
    }
    auto share = [&](int m, int a, int b) -> T {
        if constexpr (STAGE) {
            return X[m * NN + a * Nmax + b];
        } else {
            const int f1 = m < 2 ? i : m < 4 ? k : p;
            const int f2 = (m == 0 || m == 5) ? k : (m == 1 || m == 3) ? p : i;
            return CCk[beta_of(N, f1, a, f2, b)];
        }
    };

    const long long NL = (long long)N * n1;
    const long long rA = (pair_index(N, i, k) * n2 + (p - 2)) * NL * n2;
    const long long rB = (pair_index(N, i, p) * n2 + (k - 1)) * NL * n2;
    const long long rC = (pair_index(N, k, p) * n2 + i) * NL * n2;
    const int nt = (N + 3) >> 2;   // cube tiles per axis
    const int ncube = nt * nt * nt;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int stride = kSweepParts * 4;
    for (int c0 = part * 4 + wave; c0 < ncube; c0 += 2 * stride) {
        int j[2], n[2], q[2];
        bool ok[2];
        int64_t aA[2], aB[2], aC[2];
        T A0[2], B0[2], C0[2];
        for (int u = 0; u < 2; ++u) {
            const int cube = c0 + u * stride;
            const int tq = cube % nt, tn = (cube / nt) % nt, tj = cube / (nt * nt);
            j[u] = tj * 4 + (lane >> 4);
            n[u] = tn * 4 + ((lane >> 2) & 3);
            q[u] = tq * 4 + (lane & 3);
            ok[u] = cube < ncube && j[u] < N && n[u] < N && q[u] < N && j[u] != n[u] && j[u] != q[u] &&
                    n[u] != q[u];
            const int jj = j[u], nn = n[u], qq = q[u];
            const int jn = nn - (nn > jj), jq = qq - (qq > jj), nj = jj - (jj > nn), nq = qq - (qq > nn);
            aA[u] = rA + ((jj * n1 + jn) * n2 + (jq - (qq > nn)));
            aB[u] = rB + ((jj * n1 + jq) * n2 + (jn - (nn > qq)));
            aC[u] = rC + ((nn * n1 + nq) * n2 + (nj - (jj > qq)));
            if (ok[u]) {
                A0[u] = Dk[aA[u]];
                B0[u] = Dk[aB[u]];
                C0[u] = Dk[aC[u]];
            }
        }
        for (int u = 0; u < 2; ++u) {
            if (!ok[u]) continue;
            const int jj = j[u], nn = n[u], qq = q[u];
            const T mean = six_way_mean<PM>(A0[u], B0[u], C0[u], share(0, jj, nn), share(1, jj, qq), share(2, nn, jj),
                                           share(3, nn, qq), share(4, qq, jj), share(5, qq, nn));
            Dk[aA[u]] = mean;
            Dk[aB[u]] = mean;
            Dk[aC[u]] = mean;
        }
    }
}

// base[idx] with the byte offset computed in 32 bits (idx * sizeof(T) < 2^32),
// which lets the compiler address through the uniform base pointer plus a
// 32-bit lane offset instead of keeping a 64-bit address per access.
template <typename T>
__device__ __forceinline__ T& at32(T* base, unsigned idx)
{
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(T));
}

// Steps 1-3 with one workgroup per facility triple i < k < p, everything
// through LDS (for N small enough that the triple's C run, its spread-share
// tables and two location tiles of A and B fit; see sweep_triple_lds).  The
// triple's three stored runs (pair-major layout) are
//   A[L(j,n)][q'] = D_{(i,j),(k,n)}[p][q],  B[L(j,q)][n'] = D_{(i,j),(p,q)}[k][n],
//   C[L(n,q)][j'] = D_{(k,n),(p,q)}[i][j],
// L(a,b) = a (N-1) + b - [b > a], each N (N-1) (N-2) entries.  The workgroup
// reads the C run whole and the triple's six tables of spread shares, then
// for each tile of JT locations j reads the A and B rows of those j (one
// contiguous stretch each), forms the means of the tile's groups (j, n, q) as
// k_sweep_cube does, and writes the rows back; finally it writes the C run
// back.  Every HBM access is a run of consecutive entries.
//
// Every global load and store is issued unconditionally in straight-line code,
// with indices past the end clamped to the last entry (a clamped load re-reads
// it, a clamped store writes back the value it holds), so the compiler knows
// which loads are still in flight at each LDS write and waits for those alone:
// the C run, the tables and the first two tiles are all requested before
// anything is written to LDS, and while a tile is processed the rows of the
// next two tiles are in flight.
// A workgroup has NT = kTripleThreads threads, or kTripleThreadsSmall for
// instances whose triple fits it (then a CU holds more triples at once).
constexpr int kTripleThreads = 1024;
constexpr int kTripleThreadsSmall = 512;
constexpr int kTripleJT = 2;
// Entries of the C run per thread: N (N-1) (N-2) <= kTripleRunRegs * NT
// (N <= 25 in FP64, N <= 32 in FP32 at 1024 threads), loaded kTripleRunChunk
// at a time.
template <typename T>
constexpr int kTripleRunRegs = sizeof(T) == 8 ? 14 : 30;
template <typename T>
constexpr int kTripleRunChunk = sizeof(T) == 8 ? 14 : 10;

// LDS bytes of k_sweep_triple at size N with NT threads; (size_t)-1 when a
// location tile, the C run or the tables exceed what the kernel holds per
// thread.
template <typename T, int NT = kTripleThreads>
__host__ __device__ inline size_t sweep_triple_lds(int N)
{
    const size_t run = (size_t)N * (N - 1) * (N - 2);
    if ((size_t)kTripleJT * (N - 1) * (N - 2) > 2 * (size_t)NT) return (size_t)-1;
    if (run > (size_t)kTripleRunRegs<T> * NT) return (size_t)-1;
    if ((size_t)6 * N * N > 6 * (size_t)NT) return (size_t)-1;
    return (run + (size_t)6 * N * N + (size_t)2 * kTripleJT * (N - 1) * (N - 2)) * sizeof(T);
}

// Position g of a location tile (g < kTripleJT (N-1)(N-2)): the tile-local
// location jl and the compact (n', q'') of its row, which do not depend on the
// tile, so a thread computes them once per size and keeps them in registers,
// packed in one word (jl | n' << 8 | q'' << 16, each below 256).
using TileSlot = unsigned;
__device__ __forceinline__ TileSlot tile_slot(int g, int rowlen, int n2)
{
    const int jl = g / rowlen, r = g - jl * rowlen;
    const int nc = r / n2;
    return (unsigned)(jl & 255) | ((unsigned)nc << 8) | ((unsigned)(r - nc * n2) << 16);
}

// The six-way mean of the group at position g (slot sl) of the tile that
// starts at location j0, in LDS: A and B rows of the tile, the C run and the
// spread-share tables X.  Offsets are 24-bit products (all below 2^24).
template <int PM, typename T>
__device__ __forceinline__ void tile_group(T* __restrict__ As, T* __restrict__ Bs, T* __restrict__ Cs,
                                           const T* __restrict__ X, int g, TileSlot sl, int j0, int N, int n1,
                                           int n2, int rowlen, int NN)
{
    const int jl = (int)(sl & 255u), nc = (int)((sl >> 8) & 255u), qc = (int)(sl >> 16);
    const int j = j0 + jl;
    const int n = nc + (nc >= j);   // n' skips j
    const int lo = min(j, n), hi = max(j, n);
    int q = qc + (qc >= lo);        // q'' skips j and n
    q += (q >= hi);
    const int jq = q - (q > j);
    T& a = As[g];
    T& b = Bs[__umul24(jl, rowlen) + __umul24(jq, n2) + (n - (n > j) - (n > q))];
    T& c = Cs[__umul24(__umul24(n, n1) + q - (q > n), n2) + (j - (j > n) - (j > q))];
    const int jN = __umul24(j, N), nN = __umul24(n, N), qN = __umul24(q, N);
    const T mean = six_way_mean<PM>(a, b, c, X[0 * NN + jN + n], X[1 * NN + jN + q], X[2 * NN + nN + j],
                                    X[3 * NN + nN + q], X[4 * NN + qN + j], X[5 * NN + qN + n]);
    a = mean;
    b = mean;
    c = mean;
}

// Workgroup b takes triple b - pre[s] of instance ids[s] (of instance s when
// ids is null), s the last of the K prefix entries with pre[s] <= b.  The
// FP32 variants are compiled for eight waves per SIMD (64 VGPRs, two
// 1024-thread workgroups per CU); the FP64 one would spill there.
template <int PM, int NT>
__global__ __launch_bounds__(NT, PM == kPrecF64 ? 1 : 8) void k_sweep_triple(
    StoreT<PM>* __restrict__ Dd, const StoreT<PM>* __restrict__ CC, StoreT<PM>* __restrict__ B,
    const int* __restrict__ tri, const Inst* __restrict__ inst, const long long* __restrict__ pre,
    const int* __restrict__ ids, int K, const int* __restrict__ act)
{
    using T = StoreT<PM>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int s = find_seg(pre, K, (long long)blockIdx.x);
    const int id = ids ? ids[s] : s;
    if (!act[id]) return;   // whole workgroup
    const Inst I = inst[id];
    const int t = (int)((long long)blockIdx.x - pre[s]);
    if (t >= I.ntri) return;   // whole workgroup
    if (t == 0) clear_inst_B(B, I, threadIdx.x, NT);
    const int N = I.N, n1 = N - 1, n2 = N - 2;
    const int NN = N * N;
    const int run = N * n1 * n2, rowlen = n1 * n2;   // one location j: N-1 rows of N-2
    T* __restrict__ Cs = reinterpret_cast<T*>(smem);
    T* __restrict__ X = Cs + run;                    // [6][N][N]
    T* __restrict__ As = X + 6 * NN;                 // [kTripleJT][rowlen]
    T* __restrict__ Bs = As + kTripleJT * rowlen;
    const int* tr = tri + I.tri0 + 3 * t;
    const int i = tr[0], k = tr[1], p = tr[2];
    T* __restrict__ Dk = Dd + I.offD;
    const T* __restrict__ CCk = CC + I.offC;
    const long long NL = (long long)N * n1;
    T* __restrict__ gA = Dk + (pair_index(N, i, k) * n2 + (p - 2)) * NL * n2;
    T* __restrict__ gB = Dk + (pair_index(N, i, p) * n2 + (k - 1)) * NL * n2;
    T* __restrict__ gC = Dk + (pair_index(N, k, p) * n2 + i) * NL * n2;
    const int tid = threadIdx.x;
    const int ntiles = (N + kTripleJT - 1) / kTripleJT;
    // The decoded position of group tid stays in a register across the tiles.
    const TileSlot slot0 = tile_slot(tid, rowlen, n2);

    // Requests: the C run, the tables (table m holds the spread shares of the
    // facility pair (f1, f2) below; diagonal entries are never read and load
    // CCk[0]), then tiles 0 and 1.
    constexpr int RR = kTripleRunRegs<T>, RC = kTripleRunChunk<T>;
    static_assert(RR % RC == 0, "whole chunks");
    T cr[RC];
    auto loadC = [&](int c0) {
#pragma unroll
        for (int u = 0; u < RC; ++u) cr[u] = at32(gC, (unsigned)min(tid + (c0 + u) * NT, run - 1));
    };
    auto putC = [&](int c0) {
#pragma unroll
        for (int u = 0; u < RC; ++u) Cs[min(tid + (c0 + u) * NT, run - 1)] = cr[u];
    };
    loadC(0);
    T xr[6];
#pragma unroll
    for (int u = 0; u < 6; ++u) {
        const int x = min(tid + u * NT, 6 * NN - 1);
        const int m = x / NN, r = x - m * NN;
        const int a = r / N, b = r - a * N;
        const int f1 = m < 2 ? i : m < 4 ? k : p;
        const int f2 = (m == 0 || m == 5) ? k : (m == 1 || m == 3) ? p : i;
        xr[u] = CCk[a == b ? 0 : beta_of(N, f1, a, f2, b)];
    }
    auto fetch = [&](T (&ra)[2], T (&rb)[2], int tix) {
        const int j0 = min(tix, ntiles - 1) * kTripleJT;
        const int len = min(kTripleJT, N - j0) * rowlen;
        T* __restrict__ tA = gA + (long long)j0 * rowlen;
        T* __restrict__ tB = gB + (long long)j0 * rowlen;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const unsigned x = (unsigned)min(tid + u * NT, len - 1);
            ra[u] = at32(tA, x);
            rb[u] = at32(tB, x);
        }
    };
    T pa0[2], pb0[2], pa1[2], pb1[2];
    fetch(pa0, pb0, 0);
    fetch(pa1, pb1, 1);
    putC(0);
#pragma unroll
    for (int u = 0; u < 6; ++u) X[min(tid + u * NT, 6 * NN - 1)] = xr[u];
#pragma unroll
    for (int c0 = RC; c0 < RR; c0 += RC) {   // FP32 only: the rest of the run
        loadC(c0);
        putC(c0);
    }

    // One tile: its rows from registers into LDS, the rows of the tile two
    // ahead requested into the same registers, the tile's groups, the rows
    // back to HBM.
    auto tile = [&](T (&ra)[2], T (&rb)[2], int tix) {
        const int j0 = tix * kTripleJT;
        const int len = min(kTripleJT, N - j0) * rowlen;
        T* __restrict__ tA = gA + (long long)j0 * rowlen;
        T* __restrict__ tB = gB + (long long)j0 * rowlen;
        __syncthreads();   // previous tile written back (C and X in place)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int x = min(tid + u * NT, len - 1);
            As[x] = ra[u];
            Bs[x] = rb[u];
        }
        __syncthreads();
        fetch(ra, rb, tix + 2);
        // A tile has at most 2 NT groups (sweep_triple_lds): every thread
        // takes position tid, whose slot it keeps, and the first len - NT
        // threads (at most two waves) also position tid + NT, decoded here.
        if (tid < len) tile_group<PM>(As, Bs, Cs, X, tid, slot0, j0, N, n1, n2, rowlen, NN);
        if (tid + NT < len)
            tile_group<PM>(As, Bs, Cs, X, tid + NT, tile_slot(tid + NT, rowlen, n2), j0, N, n1, n2, rowlen, NN);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const unsigned x = (unsigned)min(tid + u * NT, len - 1);
            at32(tA, x) = As[x];
            at32(tB, x) = Bs[x];
        }
    };
    int tix = 0;
    for (; tix + 1 < ntiles; tix += 2) {
        tile(pa0, pb0, tix);
        tile(pa1, pb1, tix + 1);
    }
    if (tix < ntiles) tile(pa0, pb0, tix);
    __syncthreads();
    // The thread index passes through an empty asm so that these offsets are
    // computed here rather than kept in registers from the first C loop.
    int tid2 = tid;
    asm volatile("" : "+v"(tid2));
#pragma unroll
    for (int u = 0; u < RR; ++u) {
        const unsigned x = (unsigned)min(tid2 + u * NT, run - 1);
        at32(gC, x) = Cs[x];
    }
}

// k_sweep_triple as a persistent kernel: each workgroup walks the triples
// blockIdx.x, blockIdx.x + gridDim.x, ... (all triples of an instance are
// the same work, so a static walk is balanced).  As soon as a triple's C run
// and tables are in LDS, the next triple's are requested into the registers
// they came through, and the two-tiles-ahead prefetch runs on into the next
// triple's first tiles, so a triple's start overlaps the previous one's tiles.
// LDS is laid out for size Nmax, the largest instance of the launch.  Same
// arithmetic and order as k_sweep_triple.
template <typename T>
struct TripleRef {
    int N, n1, n2, NN, run, rowlen, ntiles, i, k, p;
    int live;        // the instance is active
    int first;       // the instance's first triple (its workgroup clears B)
    long long offB;  // the instance's B
    T* gA;
    T* gB;
    T* gC;
    const T* CCk;
};

template <typename T>
__device__ __forceinline__ TripleRef<T> triple_ref(T* Dd, const T* CC, const int* __restrict__ tri,
                                                   const Inst* __restrict__ inst, const long long* __restrict__ pre,
                                                   const int* __restrict__ ids, int K, long long Tg,
                                                   const int* __restrict__ act)
{
    const int s = find_seg(pre, K, Tg);
    const int id = ids ? ids[s] : s;
    const Inst I = inst[id];
    const int t = (int)(Tg - pre[s]);
    TripleRef<T> r;
    r.live = act[id];
    r.first = t == 0;
    r.offB = I.offB;
    r.N = I.N;
    r.n1 = r.N - 1;
    r.n2 = r.N - 2;
    r.NN = r.N * r.N;
    r.run = r.N * r.n1 * r.n2;
    r.rowlen = r.n1 * r.n2;
    r.ntiles = (r.N + kTripleJT - 1) / kTripleJT;
    const int* tr = tri + I.tri0 + 3 * t;
    r.i = tr[0];
    r.k = tr[1];
    r.p = tr[2];
    T* Dk = Dd + I.offD;
    const long long NL = (long long)r.N * r.n1;
    r.gA = Dk + (pair_index(r.N, r.i, r.k) * r.n2 + (r.p - 2)) * NL * r.n2;
    r.gB = Dk + (pair_index(r.N, r.i, r.p) * r.n2 + (r.k - 1)) * NL * r.n2;
    r.gC = Dk + (pair_index(r.N, r.k, r.p) * r.n2 + r.i) * NL * r.n2;
    r.CCk = CC + I.offC;
    return r;
}

template <int PM>
__global__ __launch_bounds__(kTripleThreads) void k_sweep_triple_p(StoreT<PM>* __restrict__ Dd,
                                                                   const StoreT<PM>* __restrict__ CC,
                                                                   StoreT<PM>* __restrict__ B,
                                                                   const int* __restrict__ tri,
                                                                   const Inst* __restrict__ inst,
                                                                   const long long* __restrict__ pre,
                                                                   const int* __restrict__ ids, int K,
                                                                   long long totalTri, int Nmax,
                                                                   const int* __restrict__ act)
{
    using T = StoreT<PM>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    long long Tg = blockIdx.x;
    if (Tg >= totalTri) return;   // whole workgroup
    T* __restrict__ Cs = reinterpret_cast<T*>(smem);
    T* __restrict__ X = Cs + Nmax * (Nmax - 1) * (Nmax - 2);   // [6][N][N]
    T* __restrict__ As = X + 6 * Nmax * Nmax;                  // [kTripleJT][rowlen]
    T* __restrict__ Bs = As + kTripleJT * (Nmax - 1) * (Nmax - 2);

    constexpr int RR = kTripleRunRegs<T>, RC = kTripleRunChunk<T>;
    static_assert(RR % RC == 0, "whole chunks");
    T cr[RC];
    T xr[6];
    // The run and tables of triple r go through cr and xr.
    auto loadC = [&](T* gC, int run, int c0) {
#pragma unroll
        for (int u = 0; u < RC; ++u) cr[u] = at32(gC, (unsigned)min(tid + (c0 + u) * kTripleThreads, run - 1));
    };
    auto putC = [&](int run, int c0) {
#pragma unroll
        for (int u = 0; u < RC; ++u) Cs[min(tid + (c0 + u) * kTripleThreads, run - 1)] = cr[u];
    };
    auto loadX = [&](const T* CCk, int N, int i, int k, int p) {
        const int NN = N * N;
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            const int x = min(tid + u * kTripleThreads, 6 * NN - 1);
            const int m = x / NN, rr = x - m * NN;
            const int a = rr / N, b = rr - a * N;
            const int f1 = m < 2 ? i : m < 4 ? k : p;
            const int f2 = (m == 0 || m == 5) ? k : (m == 1 || m == 3) ? p : i;
            xr[u] = CCk[a == b ? 0 : beta_of(N, f1, a, f2, b)];
        }
    };
    auto putX = [&](int N) {
#pragma unroll
        for (int u = 0; u < 6; ++u) X[min(tid + u * kTripleThreads, 6 * N * N - 1)] = xr[u];
    };
    // Rows of the tile starting at location j0 of runs (gA, gB).
    auto fetch = [&](T (&ra)[2], T (&rb)[2], T* gA, T* gB, int N, int rowlen, int j0) {
        const int len = min(kTripleJT, N - j0) * rowlen;
        T* tA = gA + (long long)j0 * rowlen;
        T* tB = gB + (long long)j0 * rowlen;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const unsigned x = (unsigned)min(tid + u * kTripleThreads, len - 1);
            ra[u] = at32(tA, x);
            rb[u] = at32(tB, x);
        }
    };

    TripleRef<T> cur = triple_ref<T>(Dd, CC, tri, inst, pre, ids, K, Tg, act);
    T pa0[2], pb0[2], pa1[2], pb1[2];
    loadC(cur.gC, cur.run, 0);
    loadX(cur.CCk, cur.N, cur.i, cur.k, cur.p);
    fetch(pa0, pb0, cur.gA, cur.gB, cur.N, cur.rowlen, 0);
    fetch(pa1, pb1, cur.gA, cur.gB, cur.N, cur.rowlen, min(kTripleJT, (cur.ntiles - 1) * kTripleJT));
    for (;;) {
        const int N = cur.N, n1 = cur.n1, n2 = cur.n2, NN = cur.NN, rowlen = cur.rowlen, ntiles = cur.ntiles;
        const int run = cur.run;
        const TileSlot slot0 = tile_slot(tid, rowlen, n2);
        T* const gA = cur.gA;
        T* const gB = cur.gB;
        T* const gC = cur.gC;
        const bool live = cur.live != 0;   // an ended instance's entries are written back unchanged
        if (live && cur.first)
            for (int e = tid; e < cur.NN; e += kTripleThreads) B[cur.offB + e] = (T)0;
        putC(run, 0);
        putX(N);
#pragma unroll
        for (int c0 = RC; c0 < RR; c0 += RC) {   // FP32 only: the rest of the run
            loadC(gC, run, c0);
            putC(run, c0);
        }
        const long long Tn = Tg + gridDim.x;
        const bool more = Tn < totalTri;
        // The next triple (when there is none, every "next" load below reads
        // one entry of this triple's runs: the code stays straight-line).
        const TripleRef<T> nxt = triple_ref<T>(Dd, CC, tri, inst, pre, ids, K, more ? Tn : Tg, act);
        T* const hA = nxt.gA;
        T* const hB = nxt.gB;
        const int hN = more ? nxt.N : 1, hrow = more ? nxt.rowlen : 1;
        const int hlast = more ? (nxt.ntiles - 1) * kTripleJT : 0;
        loadC(nxt.gC, more ? nxt.run : 1, 0);   // registers free again: the next triple's run and tables
        loadX(nxt.CCk, hN, nxt.i, nxt.k, nxt.p);
        auto tile = [&](T (&ra)[2], T (&rb)[2], int tix) {
            const int j0 = tix * kTripleJT;
            const int len = min(kTripleJT, N - j0) * rowlen;
            T* __restrict__ tA = gA + (long long)j0 * rowlen;
            T* __restrict__ tB = gB + (long long)j0 * rowlen;
            __syncthreads();   // previous tile written back (C and X in place)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int x = min(tid + u * kTripleThreads, len - 1);
                As[x] = ra[u];
                Bs[x] = rb[u];
            }
            __syncthreads();
            // Two tiles ahead: this triple's, or past its end the next one's.
            const int t2 = tix + 2;
            const bool on = t2 < ntiles;
            fetch(ra, rb, on ? gA : hA, on ? gB : hB, on ? N : hN, on ? rowlen : hrow,
                  on ? t2 * kTripleJT : min((t2 - ntiles) * kTripleJT, hlast));
            if (live && tid < len) tile_group<PM>(As, Bs, Cs, X, tid, slot0, j0, N, n1, n2, rowlen, NN);
            if (live && tid + kTripleThreads < len)
                tile_group<PM>(As, Bs, Cs, X, tid + kTripleThreads, tile_slot(tid + kTripleThreads, rowlen, n2), j0,
                               N, n1, n2, rowlen, NN);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const unsigned x = (unsigned)min(tid + u * kTripleThreads, len - 1);
                at32(tA, x) = As[x];
                at32(tB, x) = Bs[x];
            }
        };
        int tix = 0;
        for (; tix + 1 < ntiles; tix += 2) {
            tile(pa0, pb0, tix);
            tile(pa1, pb1, tix + 1);
        }
        if (tix < ntiles) tile(pa0, pb0, tix);
        __syncthreads();
        int tid2 = tid;
        asm volatile("" : "+v"(tid2));
#pragma unroll
        for (int u = 0; u < RR; ++u) {
            const unsigned x = (unsigned)min(tid2 + u * kTripleThreads, run - 1);
            at32(gC, x) = Cs[x];
        }
        if (!more) break;
        // With an odd tile count the next triple's tile 0 went into the
        // second register set.
        if (ntiles & 1) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const T ta = pa0[u], tb = pb0[u];
                pa0[u] = pa1[u];
                pb0[u] = pb1[u];
                pa1[u] = ta;
                pb1[u] = tb;
            }
        }
        __syncthreads();   // the C run has been read out of LDS
        cur = nxt;
        Tg = Tn;
    }
}

// Step 5: the complementary pair c_ijkn, c_knij (equation (10)) both become
// their mean.  One thread per C entry; the thread with i < k does the pair.
template <int PM>
__global__ __launch_bounds__(256) void k_transfer_C(StoreT<PM>* __restrict__ C, const Inst* __restrict__ inst,
                                                    const long long* __restrict__ preC, int K, long long totalC,
                                                    const int* __restrict__ act)
{
    using T = StoreT<PM>;
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= totalC) return;
    const int kk = find_seg(preC, K, x);
    if (!act[kk]) return;
    const Inst I = inst[kk];
    const int N = I.N, n1 = N - 1;
    const long long lx = x - I.offC;
    const int ij = (int)(lx / (n1 * n1));
    const int rem = (int)(lx % (n1 * n1));
    const int i = ij / N, j = ij % N;
    const int k = skip1(rem / n1, i), n = skip1(rem % n1, j);
    if (i >= k) return;
    const long long y = I.offC + beta_of(N, k, n, i, j);
    T mean;
    if constexpr (PM == kPrecF32Down)
        mean = to_float_down(div_down(add_down((double)C[x], (double)C[y]), 2.0));
    else
        mean = (T)(((double)C[x] + (double)C[y]) / 2.0);
    C[x] = mean;
    C[y] = mean;
}

// ---- FP64 certification cascade (every rounding toward -inf) ----------------
// For every permutation pi the stored state represents the objective
//   LB + sum_i b_{i pi(i)} + sum_{i!=k} c_{i pi(i) k pi(k)} + sum d_{...}.
// With m(beta) = min(0, min of block D_beta):  c~ = c + (N-2) m(beta) bounds
// the c term plus its block's N-2 entries on pi from below; likewise
// b~ = b + (N-1) min(0, min of C~_ij), and LB + N min(0, min b~) bounds the
// whole sum from below whatever the signs of the stored entries.

// One wave per stored D block of every instance: ct[beta] = c_beta +
// (N-2) min(0, min D_beta), for both blocks of the pair when HALF.  The
// blocks stored (all, or one per pair) number totalC (or totalC / 2; every
// instance's C count is a multiple of 4, so halving preC gives the prefix of
// its stored blocks).
template <typename T, bool HALF>
__global__ __launch_bounds__(256) void k_cert_D(const T* __restrict__ Dd, const T* __restrict__ C,
                                                double* __restrict__ ct, const Inst* __restrict__ inst,
                                                const long long* __restrict__ preC, int K, long long totalC)
{
    const long long x = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (x >= (HALF ? totalC / 2 : totalC)) return;
    const Inst I = inst[find_seg(preC, K, HALF ? 2 * x : x)];
    const int N = I.N, n2 = N - 2, blk = n2 * n2;
    const long long local = x - (HALF ? I.offC / 2 : I.offC);
    long long beta = local, twin = -1, base = local * I.ldD, ld = n2;
    if constexpr (HALF) {
        pair_block(N, local, &beta, &twin, &base);
        ld = (long long)N * (N - 1) * n2;
    }
    const T* __restrict__ Db = Dd + I.offD + base;
    double m = 0.0;
    for (int e = lane; e < blk; e += 64) m = __builtin_fmin(m, (double)Db[(e / n2) * ld + e % n2]);
    for (int off = 32; off > 0; off >>= 1) m = __builtin_fmin(m, __shfl_xor(m, off, 64));
    if (lane == 0) {
        const double md = mul_down((double)(N - 2), m);
        if constexpr (HALF) {
            ct[I.offC + beta] = add_down((double)C[I.offC + beta], md);
            ct[I.offC + twin] = add_down((double)C[I.offC + twin], md);
        } else {
            ct[x] = add_down((double)C[x], md);
        }
    }
}

// One wave per C block of every instance: bt[ij] = b_ij + (N-1) min(0, min C~_ij).
template <typename T>
__global__ __launch_bounds__(256) void k_cert_C(const double* __restrict__ ct, const T* __restrict__ B,
                                                double* __restrict__ bt, const Inst* __restrict__ inst,
                                                const long long* __restrict__ preB, int K, long long totalB)
{
    const long long x = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (x >= totalB) return;
    const Inst I = inst[find_seg(preB, K, x)];
    const int N = I.N, blk = (N - 1) * (N - 1);
    const double* __restrict__ cb = ct + I.offC + (x - I.offB) * blk;
    double m = 0.0;
    for (int e = lane; e < blk; e += 64) m = __builtin_fmin(m, cb[e]);
    for (int off = 32; off > 0; off >>= 1) m = __builtin_fmin(m, __shfl_xor(m, off, 64));
    if (lane == 0) bt[x] = add_down((double)B[x], mul_down((double)(N - 1), m));
}

// One wave per instance: out[k] = LB_k + N min(0, min bt over the instance).
template <typename Unused = void>
__global__ __launch_bounds__(64) void k_cert_final(const double* __restrict__ bt, const double* __restrict__ lb,
                                                   double* __restrict__ out, const Inst* __restrict__ inst)
{
    const Inst I = inst[blockIdx.x];
    const int N = I.N;
    double m = 0.0;
    for (int e = threadIdx.x; e < N * N; e += 64) m = __builtin_fmin(m, bt[I.offB + e]);
    for (int off = 32; off > 0; off >>= 1) m = __builtin_fmin(m, __shfl_xor(m, off, 64));
    if (threadIdx.x == 0) out[blockIdx.x] = add_down(lb[2 * blockIdx.x], mul_down((double)N, m));
}

}  // namespace qap
