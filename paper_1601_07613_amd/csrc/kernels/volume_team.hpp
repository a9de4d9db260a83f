// Volume term of Eq. (2), team form: TEAM lanes per element (4 for M = 4,
// 8 for M = 5), lane r < M owning conserved variable r.
//
// Lane r reads the N_p modes of its variable (the team reads the element
// record as one contiguous stretch), forms its variable's value at every
// volume point, and the team exchanges the values (DPP quad broadcasts, or
// ds_bpermute for 8-lane teams) so that every lane holds the full state.
// Every lane evaluates only its own component of the flux (the shared
// pressure and velocity, then one product per direction, no selection among
// the components); the contravariant flux and the projection onto the modes
// are lane-local (fused multiply-adds into the accumulators), and lane r
// writes its variable's N_p modes of the result.  Same formulas as
// volume_elem; the products are rounded in a different order.
#pragma once

#include <hip/hip_runtime.h>

#include "euler_dev.hpp"
#include "team.hpp"

namespace dgc_dev {

template <int DIM>
constexpr int volume_team_size() {
    return DIM + 2 <= 4 ? 4 : 8;
}

// Lanes per element of the batched volume term: the team form where it is
// the faster vector form, one work-item per element where that is faster
// (tetrahedra; f32 triangles and f32 quadrilaterals at p = 3; f64 triangles
// at p = 3; measured on 1M-element meshes).  Host and device share this rule.
__host__ __device__ constexpr int batch_volume_lanes(int dim, int np, bool f32) {
    if (dim == 3) return 1;
    const bool quad = np == 4 || np == 9 || np == 16;
    if (f32) return (quad && np != 16) ? 4 : 1;
    return np == 10 ? 1 : 4;
}

// Unroll of the point loop of the team form: a rolled loop keeps the
// registers of one point only (measured faster at every order: 58 instead of
// 122 registers at N_p = 6; two points per trip at N_p = 21).
__host__ __device__ constexpr int team_volume_unroll(int np) { return np >= 21 ? 2 : 1; }
// The same inside the fused first-color face kernel, which holds the face's
// own state besides: three points per trip at N_p = 6 (9 points; the same
// 124-126 registers, 3 % faster), elsewhere as above.
__host__ __device__ constexpr int fused_volume_unroll(int np) { return np == 6 ? 3 : team_volume_unroll(np); }

// Element k's inverse Jacobian (row-major) and sqrt(det J).
template <int DIM, class T>
__device__ __forceinline__ void load_elem_geo(int64_t k, int64_t n_elem, const double *__restrict__ elem_geo,
                                              T (&Ji)[DIM * DIM], double &sq) {
#pragma unroll
    for (int a = 0; a < DIM * DIM; ++a) Ji[a] = T(elem_geo[a * n_elem + k]);
    sq = elem_geo[DIM * DIM * n_elem + k];
}

// Lane r's share of an element's volume term from its geometry (Ji, sq and
// inv_sq = 1 / sq, the value a face record already carries): c
// holds the element's modes of variable r (zeros on lanes r >= M), out
// receives the result for variable r (all lanes of the team must call; the
// tables may live in global memory (f64) or in LDS).
template <int DIM, int NP, int QV, class T, class TAB = double, int UNR = team_volume_unroll(NP)>
__device__ __forceinline__ void volume_team_core_geo(int r, const T (&Ji)[DIM * DIM], double sq, double inv_sq,
                                                     const TAB *__restrict__ vb, const TAB *__restrict__ vd,
                                                     const T (&c)[NP], T (&out)[NP]) {
    constexpr int M = DIM + 2;
    constexpr int TEAM = volume_team_size<DIM>();
    const T isq = T(inv_sq);
    // this lane's share of the physical flux F_r(u) = a u_e / rho + [r = 1 + e] p,
    // a = u_r (+ p for the energy): 0/1 selectors fixed per lane
    const T sel_e = r == M - 1 ? T(1) : T(0);
    T sel_m[DIM];
#pragma unroll
    for (int e = 0; e < DIM; ++e) sel_m[e] = r == 1 + e ? T(1) : T(0);
    T acc[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = 0;
#pragma unroll UNR
    for (int q = 0; q < QV; ++q) {
        T t = 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) t += T(vb[q * NP + j]) * c[j];
        const T own = t * isq;
        T uq[M];
#pragma unroll
        for (int m = 0; m < M; ++m) uq[m] = team_bcast<TEAM>(own, m);
        T Fm[DIM];
        flux_component<DIM, T>(uq, own, sel_e, sel_m, Fm);
        T G[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            T g = 0;
#pragma unroll
            for (int e = 0; e < DIM; ++e) g += Ji[d * DIM + e] * Fm[e];
            G[d] = g;
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) acc[j] = dev_fma(T(vd[(d * QV + q) * NP + j]), G[d], acc[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) out[j] = acc[j] * T(sq);
}

// the same for element k, its geometry read here
template <int DIM, int NP, int QV, class T, class TAB = double, int UNR = team_volume_unroll(NP)>
__device__ __forceinline__ void volume_team_core(int64_t k, int r, int64_t n_elem,
                                                 const double *__restrict__ elem_geo, const TAB *__restrict__ vb,
                                                 const TAB *__restrict__ vd, const T (&c)[NP], T (&out)[NP]) {
    T Ji[DIM * DIM];
    double sq;
    load_elem_geo<DIM, T>(k, n_elem, elem_geo, Ji, sq);
    volume_team_core_geo<DIM, NP, QV, T, TAB, UNR>(r, Ji, sq, 1.0 / sq, vb, vd, c, out);
}

// element k, lane r of its team (all lanes of the team must call)
template <int DIM, int NP, int QV, class T, class TAB = double>
__device__ __forceinline__ void volume_team_elem(int64_t k, int r, int64_t n_elem,
                                                 const double *__restrict__ elem_geo, const TAB *__restrict__ vb,
                                                 const TAB *__restrict__ vd, const T *__restrict__ U,
                                                 T *__restrict__ rhs) {
    constexpr int M = DIM + 2;
    constexpr int REC = M * NP;
    const bool own = r < M;
    T c[NP];
    const T *u = U + (size_t)k * REC + r * NP;
#pragma unroll
    for (int j = 0; j < NP; ++j) c[j] = own ? u[j] : T(0);
    T res[NP];
    volume_team_core<DIM, NP, QV, T, TAB>(k, r, n_elem, elem_geo, vb, vd, c, res);
    if (!own) return;
    T *o = rhs + (size_t)k * REC + r * NP;
#pragma unroll
    for (int j = 0; j < NP; ++j) o[j] = res[j];
}

// Mode-team share of element k's volume term (N_p = 4, a quad of lanes, lane
// j owning mode j of every variable; c and out hold that mode of the M
// variables): the point values are quad sums of the lanes' shares, every
// lane evaluates the flux of the full state, and lane j projects onto mode j.
// (Giving each lane a quarter of the points instead avoids repeating the
// flux, but needs the whole record and all 20 projections in every lane:
// more than twice the registers.)  All four lanes of the quad must call.
template <int DIM, int NP, int QV, class T, class TAB = double>
__device__ __forceinline__ void volume_mode_team_core_geo(int j, const T (&Ji)[DIM * DIM], double sq,
                                                          double inv_sq, const TAB *__restrict__ vb,
                                                          const TAB *__restrict__ vd, const T (&c)[DIM + 2],
                                                          T (&out)[DIM + 2]) {
    static_assert(NP == 4, "mode teams need exactly four modes");
    constexpr int M = DIM + 2;
    const T isq = T(inv_sq);
    T acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0;
#pragma unroll 1
    for (int q = 0; q < QV; ++q) {
        const T t = T(vb[q * NP + j]);
        T uq[M];
#pragma unroll
        for (int m = 0; m < M; ++m) uq[m] = quad_sum(t * c[m]) * isq;
        T Fx[M * DIM];
        phys_flux<DIM, T>(uq, Fx);
        // my mode's reference gradient weights mapped to physical space once
        // per point, W_e = sum_d (J^-1)_{de} w_d, shared by the M variables
        // (3 x 3 + 5 x 3 multiply-adds instead of 5 x (3 x 3 + 3))
        T W[DIM];
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
            T g = 0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) g += Ji[d * DIM + e] * T(vd[(d * QV + q) * NP + j]);
            W[e] = g;
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
#pragma unroll
            for (int e = 0; e < DIM; ++e) acc[m] = dev_fma(W[e], Fx[m * DIM + e], acc[m]);
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) out[m] = acc[m] * T(sq);
}

// the same for element k, its geometry read here
template <int DIM, int NP, int QV, class T, class TAB = double>
__device__ __forceinline__ void volume_mode_team_core(int64_t k, int j, int64_t n_elem,
                                                      const double *__restrict__ elem_geo, const TAB *__restrict__ vb,
                                                      const TAB *__restrict__ vd, const T (&c)[DIM + 2],
                                                      T (&out)[DIM + 2]) {
    T Ji[DIM * DIM];
    double sq;
    load_elem_geo<DIM, T>(k, n_elem, elem_geo, Ji, sq);
    volume_mode_team_core_geo<DIM, NP, QV, T, TAB>(j, Ji, sq, 1.0 / sq, vb, vd, c, out);
}

template <int DIM, int NP, int QV, class T>
__global__ __launch_bounds__(256) void volume_team_kernel(int64_t n_elem, const double *__restrict__ elem_geo,
                                                          const double *__restrict__ vb,
                                                          const double *__restrict__ vd,
                                                          const T *__restrict__ U, T *__restrict__ rhs) {
    constexpr int TEAM = volume_team_size<DIM>();
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / TEAM;
    if (k >= n_elem) return;  // whole teams leave together
    volume_team_elem<DIM, NP, QV, T>(k, threadIdx.x % TEAM, n_elem, elem_geo, vb, vd, U, rhs);
}

// Mixed triangle / quadrilateral meshes (2D, N_p = (p+1)^2 slots per
// element): both kinds' volume tables are staged in LDS and each team picks
// its element's block; a triangle's tables are zero beyond its own modes.
template <int NP, int QV, class T>
__global__ __launch_bounds__(256) void volume_team_mixed_kernel(int64_t n_elem, const int8_t *__restrict__ elem_kind,
                                                                const double *__restrict__ elem_geo,
                                                                const double *__restrict__ vb2,
                                                                const double *__restrict__ vd2,
                                                                const T *__restrict__ U, T *__restrict__ rhs) {
    constexpr int TEAM = volume_team_size<2>();
    __shared__ T s_vb[2 * QV * NP];          // [kind][q][j]
    __shared__ T s_vd[2 * 2 * QV * NP];      // [kind][d][q][j]
    for (int i = threadIdx.x; i < 2 * QV * NP; i += blockDim.x) s_vb[i] = T(vb2[i]);
    for (int i = threadIdx.x; i < 4 * QV * NP; i += blockDim.x) s_vd[i] = T(vd2[i]);
    __syncthreads();
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / TEAM;
    if (k >= n_elem) return;  // whole teams leave together
    const int kind = elem_kind[k] ? 1 : 0;
    volume_team_elem<2, NP, QV, T, T>(k, threadIdx.x % TEAM, n_elem, elem_geo, s_vb + kind * QV * NP,
                                      s_vd + kind * 2 * QV * NP, U, rhs);
}

}  // namespace dgc_dev
