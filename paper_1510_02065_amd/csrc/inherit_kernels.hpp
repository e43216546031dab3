// Child nodes that inherit their parent's reduced costs (Section 6: the
// branch-and-bound tree runs the dual ascent at every node, and a node's
// children are its subproblems with one more assignment fixed).
//
// Fixing facility a at location b in a parent whose stored dual state is
// (LB, B, C, D) leaves, for every permutation pi with pi(a) = b, the parent's
// represented objective
//   LB + sum_i b_{i pi(i)} + sum_{i!=k} c_{i pi(i) k pi(k)} + sum d_{...}
// split by whether a takes part in a term.  The terms with a become terms of
// one level lower in the child, whose facilities and locations are the free
// ones in ascending order:
//   LB'             = LB + b_ab,
//   b'_ij           = b_ij + c_{ij ab} + c_{ab ij},
//   c'_{ij kn}      = c_{ij kn} + d_{ab ij kn} + d_{ij ab kn} + d_{ij kn ab},
//   d'_{ij kn pq}   = d_{ij kn pq},
// so the child's represented objective equals the parent's on every
// completion: a valid dual state for the child, and LB' >= LB when the
// parent's reduced costs are >= 0.  A level-1 child (no D) keeps the C terms
// above and drops D.
#pragma once
#include "lap_kernels.hpp"

namespace qap {

// Entry (c, lc) of block D_{(a,la),(b,lb)} of one instance (offsets within
// the instance's D; mode kAllBlocks or kHalfStore).
__device__ __forceinline__ long long d_entry(int N, int mode, long long ldD, int a, int la, int b, int lb, int c,
                                             int lc)
{
    if (mode == kAllBlocks) return beta_of(N, a, la, b, lb) * ldD + entry_of(N, a, la, b, lb, c, lc);
    if (a > b) {   // the stored block of the pair is the one with the smaller facility first
        const int t = a, tl = la;
        a = b;
        la = lb;
        b = t;
        lb = tl;
    }
    return pair_row(N, a, la, b, lb, drop2(c, a, b)) + drop2(lc, la, lb);
}

// Description of the children of one parent instance, shared by the kernels.
template <typename T>
struct ChildSrc {
    const T* B;          // parent instance's B (N x N)
    const T* C;          // parent instance's C
    const T* D;          // parent instance's D, nullptr for a level-1 parent
    const double* lb;    // parent instance's (LB, LB')
    int N;               // parent size
    int mode;            // parent D storage (kAllBlocks / kHalfStore)
    long long ldD;       // parent block stride (kAllBlocks)
    const int* fix;      // fix[2c], fix[2c+1]: facility and location child c fixes
};

// One thread per child B entry: b'_ij, and LB' from the thread of entry 0.
template <int PM>
__global__ __launch_bounds__(256) void k_child_B(ChildSrc<StoreT<PM>> src, StoreT<PM>* __restrict__ B,
                                                 double* __restrict__ lb, const Inst* __restrict__ inst, int K)
{
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int M = src.N - 1;
    if (x >= (long long)K * M * M) return;
    const int c = (int)(x / (M * M));
    const int e = (int)(x - (long long)c * M * M);
    const int a = src.fix[2 * c], b = src.fix[2 * c + 1];
    const int i = skip1(e / M, a), j = skip1(e % M, b);
    const int N = src.N;
    const double v0 = (double)src.B[i * N + j];
    const double v1 = (double)src.C[beta_of(N, i, j, a, b)];
    const double v2 = (double)src.C[beta_of(N, a, b, i, j)];
    const Inst I = inst[c];
    if constexpr (PM == kPrecF32Down)
        B[I.offB + e] = to_float_down(add_down(add_down(v0, v1), v2));
    else
        B[I.offB + e] = (StoreT<PM>)((v0 + v1) + v2);
    if (e == 0) {
        const double L = src.lb[0];
        const double bab = (double)src.B[a * N + b];
        lb[2 * c] = PM == kPrecF32Down ? add_down(L, bab) : L + bab;
        lb[2 * c + 1] = 0.0;
    }
}

// One thread per child C entry: c'_{ij kn}.
template <int PM>
__global__ __launch_bounds__(256) void k_child_C(ChildSrc<StoreT<PM>> src, StoreT<PM>* __restrict__ C,
                                                 const Inst* __restrict__ inst, int K)
{
    const int M = src.N - 1, m1 = M - 1;
    const long long per = (long long)M * M * m1 * m1;
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (long long)K * per) return;
    const int c = (int)(x / per);
    const long long e = x - (long long)c * per;
    const int a = src.fix[2 * c], b = src.fix[2 * c + 1];
    const int ij = (int)(e / (m1 * m1)), rem = (int)(e % (m1 * m1));
    const int ic = ij / M, jc = ij % M;
    const int kc = skip1(rem / m1, ic), nc = skip1(rem % m1, jc);   // child indices
    const int i = skip1(ic, a), j = skip1(jc, b), k = skip1(kc, a), n = skip1(nc, b);
    const int N = src.N;
    const double v0 = (double)src.C[beta_of(N, i, j, k, n)];
    double v1 = 0.0, v2 = 0.0, v3 = 0.0;
    if (src.D) {
        v1 = (double)src.D[d_entry(N, src.mode, src.ldD, a, b, i, j, k, n)];
        v2 = (double)src.D[d_entry(N, src.mode, src.ldD, i, j, a, b, k, n)];
        v3 = (double)src.D[d_entry(N, src.mode, src.ldD, i, j, k, n, a, b)];
    }
    const Inst I = inst[c];
    if constexpr (PM == kPrecF32Down)
        C[I.offC + e] = to_float_down(add_down(add_down(add_down(v0, v1), v2), v3));
    else
        C[I.offC + e] = (StoreT<PM>)(((v0 + v1) + v2) + v3);
}

// One thread per stored child D entry (level-2 children of a level-2
// parent; child storage `cmode`, the parent's): d'_{ij kn pq} = d_{ij kn pq}.
template <int PM>
__global__ __launch_bounds__(256) void k_child_D(ChildSrc<StoreT<PM>> src, StoreT<PM>* __restrict__ D,
                                                 const Inst* __restrict__ inst, int K, long long per, int cmode)
{
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (long long)K * per) return;
    const int c = (int)(x / per);
    const long long e = x - (long long)c * per;
    const int a = src.fix[2 * c], b = src.fix[2 * c + 1];
    const int M = src.N - 1, m1 = M - 1, m2 = M - 2;
    const Inst I = inst[c];
    int ic, jc, kc, nc, pr, qr;   // child block (ic,jc,kc,nc), compact row and column
    long long off;
    if (cmode == kAllBlocks) {
        const long long blk = (long long)m2 * m2;
        const long long beta = e / I.ldD;
        const int w = (int)(e - beta * I.ldD);
        if (w >= blk) return;   // block padding
        const int ij = (int)(beta / (m1 * m1)), rem = (int)(beta % (m1 * m1));
        ic = ij / M;
        jc = ij % M;
        kc = skip1(rem / m1, ic);
        nc = skip1(rem % m1, jc);
        pr = w / m2;
        qr = w % m2;
        off = e;
    } else {
        // pair-major: ((P(ic,kc) m2 + pr) M m1 + L(jc,nc)) m2 + qr
        qr = (int)(e % m2);
        long long r = e / m2;
        const int L = (int)(r % ((long long)M * m1));
        r /= (long long)M * m1;
        pr = (int)(r % m2);
        int P = (int)(r / m2);
        int a0 = 0;
        while (P >= m1 - a0) {
            P -= m1 - a0;
            ++a0;
        }
        ic = a0;
        kc = a0 + 1 + P;
        jc = L / m1;
        nc = skip1(L % m1, jc);
        off = e;
    }
    const int pc = skip2(pr, min(ic, kc), max(ic, kc));
    const int qc = skip2(qr, min(jc, nc), max(jc, nc));
    const int i = skip1(ic, a), j = skip1(jc, b), k = skip1(kc, a), n = skip1(nc, b);
    const int p = skip1(pc, a), q = skip1(qc, b);
    D[I.offD + off] = src.D[d_entry(src.N, src.mode, src.ldD, i, j, k, n, p, q)];
}

// Level-1 certification: no D, so c~ = c.
template <typename T>
__global__ __launch_bounds__(256) void k_cert_noD(const T* __restrict__ C, double* __restrict__ ct, long long totalC)
{
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < totalC) ct[x] = (double)C[x];
}

}  // namespace qap
