// Wavefront primitives for the assignment kernels on gfx950 (wave64): ballot,
// cross-lane moves (DPP, permlane swaps), the wave-local LDS ordering fence
// and NaN-free minima.  The solver built on them is in lap_slots.hpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlt2_kernels.hpp"

namespace qap {

// Wave-wide ballot of a predicate; taking a bool (not an int as __ballot
// does) lets the compiler use the comparison's lane mask directly.
__device__ __forceinline__ unsigned long long ballot64(bool pred) { return __builtin_amdgcn_ballot_w64(pred); }
// This lane's bit of a wave-uniform lane mask.  A predicate kept as such a
// mask combines with others on the scalar unit, and a ballot of it costs no
// vector instructions (a ballot of a combined bool is rebuilt lane by lane).
__device__ __forceinline__ bool lane_bit(unsigned long long mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }

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
enum DppCtrl : int { kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140 };

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

}  // namespace qap
