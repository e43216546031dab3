// Cost-concentration kernels (Section 4.1 of arXiv 1510.02065): one wave per
// workgroup, 64/SEG assignment problems per wave, each staged in LDS.
#pragma once
#include "lap_wave.hpp"

namespace qap {

// Family kernel: blocks[b*bstride ...] (n x n, row-major, contiguous) for
// b < nblocks.  parent[b] += S, the block is replaced by its residual, and
// values[b] = S when values is not null.  Used for D -> C (n = N-2, parent C)
// and C -> B (n = N-1, parent B).
template <typename T, int SEG>
__global__ __launch_bounds__(64) void k_lap_family(T* __restrict__ blocks, int64_t bstride, int n,
                                                   int64_t nblocks, T* __restrict__ parent,
                                                   double* __restrict__ values)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int LPW = 64 / SEG;
    const int seg = threadIdx.x / SEG;
    const int lane = threadIdx.x & (SEG - 1);
    const int64_t b = (int64_t)blockIdx.x * LPW + seg;
    const bool active = b < nblocks;
    const size_t sb = SegLds<T, SEG>::bytes(n);
    unsigned char* base = smem + seg * sb;
    T* Ms = reinterpret_cast<T*>(base);
    const size_t mb = SegLds<T, SEG>::mat_bytes(n);
    int* sig_s = reinterpret_cast<int*>(base + mb);
    double* va_s = reinterpret_cast<double*>(base + mb + SEG * sizeof(int));
    double* vb_s = va_s + SEG;

    T* blk = blocks + (active ? b : 0) * bstride;
    if (active)
        for (int e = lane; e < n * n; e += SEG) Ms[e] = blk[e];
    __syncthreads();
    const double S = lap_concentrate_seg<T, SEG>(Ms, active ? n : 0, sig_s, va_s, vb_s,
                                                 active ? blk : nullptr, nullptr, nullptr);
    if (active && lane == 0) {
        if constexpr (sizeof(T) == 8)
            parent[b] = parent[b] + S;
        else
            parent[b] = to_float_down(add_down((double)parent[b], S));
        if (values) values[b] = S;
    }
}

// B -> LB' (steps 7-8): the single N x N problem over B; LB += LB' in FP64.
// lb[0] = LB, lb[1] = LB'.  The trace gets (LB, LB') at position
// (*counter)++ when below trace_cap.
template <typename T, int SEG>
__global__ __launch_bounds__(64) void k_lap_B(T* __restrict__ B, int n, double* __restrict__ lb,
                                              double* __restrict__ trace,
                                              long long* __restrict__ counter, long long trace_cap,
                                              double* __restrict__ values)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int seg = threadIdx.x / SEG;
    const int lane = threadIdx.x & (SEG - 1);
    const bool active = seg == 0;
    const size_t sb = SegLds<T, SEG>::bytes(n);
    unsigned char* base = smem + seg * sb;
    T* Ms = reinterpret_cast<T*>(base);
    const size_t mb = SegLds<T, SEG>::mat_bytes(n);
    int* sig_s = reinterpret_cast<int*>(base + mb);
    double* va_s = reinterpret_cast<double*>(base + mb + SEG * sizeof(int));
    double* vb_s = va_s + SEG;
    if (active)
        for (int e = lane; e < n * n; e += SEG) Ms[e] = B[e];
    __syncthreads();
    const double S = lap_concentrate_seg<T, SEG>(Ms, active ? n : 0, sig_s, va_s, vb_s,
                                                 active ? B : nullptr, nullptr, nullptr);
    if (active && lane == 0) {
        // FP32 certified mode accumulates the bound rounding toward -inf.
        const double L = (sizeof(T) == 4) ? add_down(lb[0], S) : lb[0] + S;
        lb[0] = L;
        lb[1] = S;
        if (values) values[0] = S;
        if (counter) {
            const long long t = *counter;
            if (t < trace_cap) {
                trace[2 * t] = L;
                trace[2 * t + 1] = S;
            }
            *counter = t + 1;
        }
    }
}

// Generic batch (qap_lap_solve): problem b has size n[b] (<= SEG, else its
// value is NaN and nothing else is written), matrix at cost + mat_off[b],
// vectors at vec_off[b].
template <typename T, int SEG>
__global__ __launch_bounds__(64) void k_lap_batch(int batch, const int32_t* __restrict__ nv,
                                                  const int64_t* __restrict__ mat_off,
                                                  const int64_t* __restrict__ vec_off,
                                                  T* __restrict__ cost, double* __restrict__ value,
                                                  T* __restrict__ duals, int32_t* __restrict__ assign,
                                                  int write_residual)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int LPW = 64 / SEG;
    const int seg = threadIdx.x / SEG;
    const int lane = threadIdx.x & (SEG - 1);
    const int64_t b = (int64_t)blockIdx.x * LPW + seg;
    int n = (b < batch) ? nv[b] : 0;
    const bool bad = n < 0 || n > SEG;
    if (bad) n = 0;
    const size_t sb = SegLds<T, SEG>::bytes(SEG);
    unsigned char* base = smem + seg * sb;
    T* Ms = reinterpret_cast<T*>(base);
    const size_t mb = SegLds<T, SEG>::mat_bytes(SEG);
    int* sig_s = reinterpret_cast<int*>(base + mb);
    double* va_s = reinterpret_cast<double*>(base + mb + SEG * sizeof(int));
    double* vb_s = va_s + SEG;
    T* mat = (b < batch && !bad) ? cost + mat_off[b] : nullptr;
    const int64_t vo = (b < batch && !bad) ? vec_off[b] : 0;
    for (int e = lane; e < n * n; e += SEG) Ms[e] = mat[e];
    __syncthreads();
    const double S = lap_concentrate_seg<T, SEG>(
        Ms, n, sig_s, va_s, vb_s, (write_residual && n > 0) ? mat : nullptr,
        (duals && n > 0) ? duals + 4 * vo : nullptr, (assign && n > 0) ? assign + vo : nullptr);
    if (b < batch && lane == 0) value[b] = bad ? __builtin_nan("") : S;
}

}  // namespace qap
