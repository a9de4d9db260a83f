// Exchanges inside a team of consecutive lanes of a wave: broadcast of one
// lane's value and the order-fixed sum over a quad of four lanes.
#pragma once

#include <hip/hip_runtime.h>

namespace dgc_dev {

// Value of lane k of the caller's team (TEAM consecutive lanes).  Teams of
// four use a DPP quad broadcast (a register move, no LDS traffic); wider
// teams use ds_bpermute through __shfl.
template <int TEAM>
__device__ __forceinline__ int team_bcast_i(int v, int k) {
    if constexpr (TEAM == 4) {
        switch (k) {
            case 0: return __builtin_amdgcn_mov_dpp(v, 0x00, 0xF, 0xF, false);
            case 1: return __builtin_amdgcn_mov_dpp(v, 0x55, 0xF, 0xF, false);
            case 2: return __builtin_amdgcn_mov_dpp(v, 0xAA, 0xF, 0xF, false);
            default: return __builtin_amdgcn_mov_dpp(v, 0xFF, 0xF, 0xF, false);
        }
    } else {
        return __shfl(v, k, TEAM);
    }
}

template <int TEAM>
__device__ __forceinline__ double team_bcast(double v, int k) {
    const int lo = team_bcast_i<TEAM>(__double2loint(v), k);
    const int hi = team_bcast_i<TEAM>(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

template <int TEAM>
__device__ __forceinline__ float team_bcast(float v, int k) {
    return __int_as_float(team_bcast_i<TEAM>(__float_as_int(v), k));
}

// Sum over the 4 lanes of a quad (butterfly with DPP quad permutations);
// every lane of the quad gets the same, order-independent result
// ((v0 + v1) + (v2 + v3)).
__device__ __forceinline__ int quad_xor1_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ int quad_xor2_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false); }

__device__ __forceinline__ double quad_xor1(double v) {
    return __hiloint2double(quad_xor1_i(__double2hiint(v)), quad_xor1_i(__double2loint(v)));
}
__device__ __forceinline__ double quad_xor2(double v) {
    return __hiloint2double(quad_xor2_i(__double2hiint(v)), quad_xor2_i(__double2loint(v)));
}
__device__ __forceinline__ float quad_xor1(float v) { return __int_as_float(quad_xor1_i(__float_as_int(v))); }
__device__ __forceinline__ float quad_xor2(float v) { return __int_as_float(quad_xor2_i(__float_as_int(v))); }

template <class T>
__device__ __forceinline__ T quad_sum(T v) {
    v = v + quad_xor1(v);
    return v + quad_xor2(v);
}

}  // namespace dgc_dev
