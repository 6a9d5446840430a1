// step_common.hpp -- device pieces shared by the LF block-update kernels:
// the Rusanov flux of a face from its two reconstructed states.
#pragma once

#include "physics.hpp"

namespace mapk {

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
