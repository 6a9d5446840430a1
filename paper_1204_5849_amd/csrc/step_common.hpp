// step_common.hpp -- device pieces shared by the block-update kernels: the
// WENO face states and the Rusanov flux of a face from its two reconstructed
// states.
#pragma once

#include "physics.hpp"

namespace mapk {

// WENO face states of a cell from its neighbours um, up along one dimension
// (Sec. 3.3, component-wise, third order): L = u^-_{i+1/2} and
// R = u^+_{i-1/2}.  The smoothness weights are a = 1/s^2 with
// s = eps + (difference)^2, eps = 1e-12; multiplying numerator and
// denominator by s_-^2 s_+^2 leaves one division per state:
//   L = (2 s_-^2 w + s_+^2 v) / (2 s_-^2 + s_+^2),  w = (u0 + up)/2, v = (3 u0 - um)/2
//   R = (s_-^2 w' + 2 s_+^2 v') / (s_-^2 + 2 s_+^2), w' = (3 u0 - up)/2, v' = (u0 + um)/2
// In FP32 both s are first scaled by one power of two (exact), so that their
// squares neither overflow nor both underflow.
template <typename T>
__device__ __forceinline__ void weno_pair(T um, T u0, T up, T &L, T &R)
{
    const T dm = u0 - um, dp = up - u0;
    T sm = T(1e-12) + dm * dm, sp = T(1e-12) + dp * dp;
    if constexpr (sizeof(T) == 4) {
        const int e = __builtin_amdgcn_frexp_expf(sm > sp ? sm : sp);
        sm = __builtin_amdgcn_ldexpf(sm, -e);
        sp = __builtin_amdgcn_ldexpf(sp, -e);
    }
    const T qm = sm * sm, qp = sp * sp;
    const T h = T(0.5);
    L = Num<T>::div(T(2) * qm * (h * (u0 + up)) + qp * (h * (T(3) * u0 - um)), T(2) * qm + qp);
    R = Num<T>::div(qm * (h * (T(3) * u0 - up)) + T(2) * qp * (h * (u0 + um)), qm + T(2) * qp);
}

// Rusanov flux (Equ:LFFlux) across a face normal to dimension d, with alpha
// = max of the two fast speeds for the MHD components and c_h for the GLM
// pair (B_d, psi); the pressures of both states are given (computed once
// when the states were formed).  d may differ between lanes (see flux_sel).
template <typename T>
__device__ __forceinline__ void rusanov_sel(const T L[NV], T pL, const T R[NV], T pR, int d,
                                            T gamma, T ch, T ch2, T f[NV])
{
    Prim<T> wL, wR;
    wL.ir = Num<T>::rcp(L[RHO]);
    wL.vx = L[MX] * wL.ir;
    wL.vy = L[MY] * wL.ir;
    wL.vz = L[MZ] * wL.ir;
    wL.bb = L[BX] * L[BX] + L[BY] * L[BY] + L[BZ] * L[BZ];
    wL.p = pL;
    wR.ir = Num<T>::rcp(R[RHO]);
    wR.vx = R[MX] * wR.ir;
    wR.vy = R[MY] * wR.ir;
    wR.vz = R[MZ] * wR.ir;
    wR.bb = R[BX] * R[BX] + R[BY] * R[BY] + R[BZ] * R[BZ];
    wR.p = pR;
    T FL[NV], FR[NV];
    flux_sel(L, wL, d, ch2, FL);
    flux_sel(R, wR, d, ch2, FR);
    const T sL = speed_sel(L, wL, d, gamma), sR = speed_sel(R, wR, d, gamma);
    const T al = sL > sR ? sL : sR;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        const T ak = (k == BX + d || k == PSI) ? ch : al;
        f[k] = T(0.5) * (FL[k] + FR[k]) - T(0.5) * ak * (R[k] - L[k]);
    }
}

template <int D, typename T>
__device__ __forceinline__ void rusanov_p(const T L[NV], T pL, const T R[NV], T pR, T gamma,
                                          T ch, T ch2, T f[NV])
{
    rusanov_sel(L, pL, R, pR, D, gamma, ch, ch2, f);
}

}  // namespace mapk
