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

// Block number of D_{(a,la),(b,lb)} (= position of c_{a la b lb} in C).
__device__ __forceinline__ int64_t beta_of(int N, int a, int la, int b, int lb) {
    const int n1 = N - 1;
    return ((int64_t)(a * N + la) * n1 + drop1(b, a)) * n1 + drop1(lb, la);
}
// Offset of d_{(a,la),(b,lb),(c,lc)} inside block beta_of(a,la,b,lb).
__device__ __forceinline__ int entry_of(int N, int a, int la, int b, int lb, int c, int lc) {
    return drop2(c, a, b) * (N - 2) + drop2(lc, la, lb);
}

// Initial dual (the lines of Algorithm 1 before its loop):
//   b_ij = f_ii d_jj (+ B0_ij), c_ijkn = f_ik d_jn.
template <typename T>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ F, const double* __restrict__ Dm,
                                              const double* __restrict__ B0, T* __restrict__ B,
                                              T* __restrict__ C, int N)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n1 = N - 1;
    const int64_t nC = (int64_t)N * N * n1 * n1;
    if (x < (int64_t)N * N) {
        const int i = (int)(x / N), j = (int)(x % N);
        double b = F[i * N + i] * Dm[j * N + j];
        if (B0) b = b + B0[x];
        B[x] = (T)b;
    }
    if (x < nC) {
        const int ij = (int)(x / (n1 * n1));
        const int rem = (int)(x % (n1 * n1));
        const int i = ij / N, j = ij % N;
        const int k = skip1(rem / n1, i), n = skip1(rem % n1, j);
        C[x] = (T)(F[i * N + k] * Dm[j * N + n]);
    }
}

// Steps 1-2 precomputation: the amount each entry of block D_beta receives,
//   CC_beta = (c_beta + b_ij / (N-1)) / (N-2),
// after which c is cleared (B is cleared by the sweep, which no longer reads it).
template <typename T>
__global__ __launch_bounds__(256) void k_spread_prep(T* __restrict__ C, const T* __restrict__ B,
                                                     T* __restrict__ CC, int N)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n1 = N - 1;
    if (x >= (int64_t)N * N * n1 * n1) return;
    const int ij = (int)(x / (n1 * n1));
    const T share_b = B[ij] / (T)(N - 1);
    const T c = C[x] + share_b;
    CC[x] = c / (T)(N - 2);
    C[x] = (T)0;
}

// Steps 1-3 on D: every entry gets its block's spread share, then each group
// of six complementary coefficients (equation (11)) is replaced by its mean.
// One thread per group.  A group is an unordered triple of (facility,
// location) pairs; it is enumerated as a facility triple i < k < p (from
// `tri`) times an ordered location triple (j, n, q) of distinct locations,
// with q varying fastest so that the members (P1 P2 P3) and (P2 P1 P3) are
// read and written contiguously.  With P1=(i,j), P2=(k,n), P3=(p,q) the six
// members are summed in lexicographic order of the permutation of
// (P1, P2, P3), so the result is the same bits on every run.
template <typename T>
__global__ __launch_bounds__(256) void k_sweep(T* __restrict__ Dd, const T* __restrict__ CC,
                                               T* __restrict__ B, const int* __restrict__ tri,
                                               int N, int64_t ldD, int64_t ngroups)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < (int64_t)N * N) B[g] = (T)0;
    if (g >= ngroups) return;
    const int n1 = N - 1, n2 = N - 2;
    const int64_t L = (int64_t)N * n1 * n2;
    const int t = (int)(g / L);
    const int loc = (int)(g % L);
    const int qq = loc % n2;
    const int rest = loc / n2;
    const int j = rest / n1;
    const int n = skip1(rest % n1, j);
    const int q = skip2(qq, min(j, n), max(j, n));
    const int i = tri[3 * t], k = tri[3 * t + 1], p = tri[3 * t + 2];

    const int64_t b0 = beta_of(N, i, j, k, n), b1 = beta_of(N, i, j, p, q);
    const int64_t b2 = beta_of(N, k, n, i, j), b3 = beta_of(N, k, n, p, q);
    const int64_t b4 = beta_of(N, p, q, i, j), b5 = beta_of(N, p, q, k, n);
    const int64_t a0 = b0 * ldD + entry_of(N, i, j, k, n, p, q);
    const int64_t a1 = b1 * ldD + entry_of(N, i, j, p, q, k, n);
    const int64_t a2 = b2 * ldD + entry_of(N, k, n, i, j, p, q);
    const int64_t a3 = b3 * ldD + entry_of(N, k, n, p, q, i, j);
    const int64_t a4 = b4 * ldD + entry_of(N, p, q, i, j, k, n);
    const int64_t a5 = b5 * ldD + entry_of(N, p, q, k, n, i, j);

    const T m0 = Dd[a0] + CC[b0];
    const T m1 = Dd[a1] + CC[b1];
    const T m2 = Dd[a2] + CC[b2];
    const T m3 = Dd[a3] + CC[b3];
    const T m4 = Dd[a4] + CC[b4];
    const T m5 = Dd[a5] + CC[b5];
    T s = m0;
    s += m1;
    s += m2;
    s += m3;
    s += m4;
    s += m5;
    const T mean = s / (T)6;
    Dd[a0] = mean;
    Dd[a1] = mean;
    Dd[a2] = mean;
    Dd[a3] = mean;
    Dd[a4] = mean;
    Dd[a5] = mean;
}

// Step 5: the complementary pair c_ijkn, c_knij (equation (10)) both become
// their mean.  One thread per entry; the thread with i < k does the pair.
template <typename T>
__global__ __launch_bounds__(256) void k_transfer_C(T* __restrict__ C, int N)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n1 = N - 1;
    if (x >= (int64_t)N * N * n1 * n1) return;
    const int ij = (int)(x / (n1 * n1));
    const int rem = (int)(x % (n1 * n1));
    const int i = ij / N, j = ij % N;
    const int k = skip1(rem / n1, i), n = skip1(rem % n1, j);
    if (i >= k) return;
    const int64_t y = beta_of(N, k, n, i, j);
    const T mean = (C[x] + C[y]) / (T)2;
    C[x] = mean;
    C[y] = mean;
}

}  // namespace qap
