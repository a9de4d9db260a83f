// Device-side Euler physics: Rusanov flux along a unit normal and the
// reflective-wall mirror state.  Ideal gas, gamma = 1.4, conserved variables
// (rho, rho u[, rho v[, rho w]], E).
#pragma once

#include <hip/hip_runtime.h>

namespace dgc_dev {

constexpr double kGamma = 1.4;

template <class T>
__device__ __forceinline__ T dev_sqrt(T x);
template <>
__device__ __forceinline__ double dev_sqrt<double>(double x) { return __builtin_sqrt(x); }
template <>
__device__ __forceinline__ float dev_sqrt<float>(float x) { return __builtin_sqrtf(x); }

// a * b + c with one rounding, in the precision of the operands
__device__ __forceinline__ double dev_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float dev_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// 1/x: the hardware reciprocal refined by one Newton-Raphson step,
// r <- r + r (1 - x r), which leaves it within about an ulp of the rounded
// quotient (3 instructions instead of the ~10 of an IEEE division; the
// fluxes divide by rho at every quadrature point)
template <class T>
__device__ __forceinline__ T dev_recip(T x);
template <>
__device__ __forceinline__ double dev_recip<double>(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
template <>
__device__ __forceinline__ float dev_recip<float>(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}

// F*(uL, uR, n) = (F(uL).n + F(uR).n)/2 - lambda (uR - uL)/2,
// lambda = max(|uL.n| + cL, |uR.n| + cR), c = sqrt(gamma p / rho).
template <int DIM, class T>
__device__ __forceinline__ void rusanov(const T *uL, const T *uR, const T *n, T *F) {
    constexpr int M = DIM + 2;
    const T g1 = T(kGamma - 1.0);
    const T irl = dev_recip<T>(uL[0]), irr = dev_recip<T>(uR[0]);
    T unl = 0, unr = 0, kel = 0, ker = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        unl += uL[1 + d] * n[d];
        unr += uR[1 + d] * n[d];
        kel += uL[1 + d] * uL[1 + d];
        ker += uR[1 + d] * uR[1 + d];
    }
    unl *= irl;
    unr *= irr;
    const T pl = g1 * (uL[M - 1] - T(0.5) * kel * irl);
    const T pr = g1 * (uR[M - 1] - T(0.5) * ker * irr);
    const T cl = dev_sqrt<T>(T(kGamma) * pl * irl);
    const T cr = dev_sqrt<T>(T(kGamma) * pr * irr);
    const T al = (unl < 0 ? -unl : unl) + cl;
    const T ar = (unr < 0 ? -unr : unr) + cr;
    const T lam = al > ar ? al : ar;
    F[0] = T(0.5) * (uL[0] * unl + uR[0] * unr) - T(0.5) * lam * (uR[0] - uL[0]);
#pragma unroll
    for (int d = 0; d < DIM; ++d)
        F[1 + d] = T(0.5) * (uL[1 + d] * unl + uR[1 + d] * unr + (pl + pr) * n[d]) - T(0.5) * lam * (uR[1 + d] - uL[1 + d]);
    F[M - 1] = T(0.5) * ((uL[M - 1] + pl) * unl + (uR[M - 1] + pr) * unr) - T(0.5) * lam * (uR[M - 1] - uL[M - 1]);
}

// mirror state across a wall: momentum reflected, density and energy kept
template <int DIM, class T>
__device__ __forceinline__ void wall_ghost(const T *u, const T *n, T *g) {
    constexpr int M = DIM + 2;
    T mn = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) mn += u[1 + d] * n[d];
    g[0] = u[0];
#pragma unroll
    for (int d = 0; d < DIM; ++d) g[1 + d] = u[1 + d] - T(2) * mn * n[d];
    g[M - 1] = u[M - 1];
}

// physical flux F(u) in direction e for all variables: out[m]
template <int DIM, class T>
__device__ __forceinline__ void phys_flux(const T *u, T *Fx /* [M][DIM] */) {
    constexpr int M = DIM + 2;
    const T ir = dev_recip<T>(u[0]);
    T ke = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) ke += u[1 + d] * u[1 + d];
    const T p = T(kGamma - 1.0) * (u[M - 1] - T(0.5) * ke * ir);
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
        const T ve = u[1 + e] * ir;
        Fx[0 * DIM + e] = u[1 + e];
#pragma unroll
        for (int d = 0; d < DIM; ++d) Fx[(1 + d) * DIM + e] = u[1 + d] * ve + (d == e ? p : T(0));
        Fx[(M - 1) * DIM + e] = (u[M - 1] + p) * ve;
    }
}

// Component r of the physical flux of the full state u, for the lane that
// owns variable r (own = u[r]): F_r(u)_e = a u_{1+e} / rho + [r = 1 + e] p
// with a = u_r, plus p for the energy; sel_e = [r = M - 1] and
// sel_m[e] = [r = 1 + e] as 0/1 values.  The mass component comes out as
// rho (u_{1+e} / rho) instead of u_{1+e} itself (a rounding apart).
template <int DIM, class T>
__device__ __forceinline__ void flux_component(const T *u, T own, T sel_e, const T *sel_m, T *Fr /* [DIM] */) {
    constexpr int M = DIM + 2;
    const T ir = dev_recip<T>(u[0]);
    T ke = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) ke += u[1 + d] * u[1 + d];
    const T p = T(kGamma - 1.0) * (u[M - 1] - T(0.5) * ke * ir);
    const T a = own + sel_e * p;
#pragma unroll
    for (int e = 0; e < DIM; ++e) Fr[e] = a * (u[1 + e] * ir) + sel_m[e] * p;
}

// Component r of the Rusanov flux (same formula as rusanov) for the lane
// that owns variable r: ownL / ownR are u_L[r] / u_R[r], n_r = n[r - 1] for
// a momentum lane and 0 otherwise, sel_e = [r = M - 1].  Summed in the same
// order as rusanov.
template <int DIM, class T>
__device__ __forceinline__ T rusanov_component(const T *uL, const T *uR, const T *n, T ownL, T ownR, T n_r,
                                               T sel_e) {
    constexpr int M = DIM + 2;
    const T g1 = T(kGamma - 1.0);
    const T irl = dev_recip<T>(uL[0]), irr = dev_recip<T>(uR[0]);
    T unl = 0, unr = 0, kel = 0, ker = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        unl += uL[1 + d] * n[d];
        unr += uR[1 + d] * n[d];
        kel += uL[1 + d] * uL[1 + d];
        ker += uR[1 + d] * uR[1 + d];
    }
    unl *= irl;
    unr *= irr;
    const T pl = g1 * (uL[M - 1] - T(0.5) * kel * irl);
    const T pr = g1 * (uR[M - 1] - T(0.5) * ker * irr);
    const T cl = dev_sqrt<T>(T(kGamma) * pl * irl);
    const T cr = dev_sqrt<T>(T(kGamma) * pr * irr);
    const T al = (unl < 0 ? -unl : unl) + cl;
    const T ar = (unr < 0 ? -unr : unr) + cr;
    const T lam = al > ar ? al : ar;
    const T aL = ownL + sel_e * pl, aR = ownR + sel_e * pr;
    return T(0.5) * (aL * unl + aR * unr + (pl + pr) * n_r) - T(0.5) * lam * (ownR - ownL);
}

}  // namespace dgc_dev
