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

// HLLC flux (the solver the paper names for MHD, Gurski's construction with
// the intermediate states of Li's HLLC for MHD) across a face normal to d.
// The GLM pair (B_d, psi) takes the exact upwind flux of its linear system:
// interface values B_m = (B_dL + B_dR)/2 - (psi_R - psi_L)/(2 c_h) and
// psi_m = (psi_L + psi_R)/2 - c_h (B_dR - B_dL)/2, fluxes psi_m and
// c_h^2 B_m.  Both states then take B_d = B_m (their gas pressures follow,
// e unchanged), and the other components get the HLLC fan: outer speeds
// S_L = min(v_L, v_R) - max(c_fL, c_fR), S_R = max(v_L, v_R) + max(c_fL, c_fR);
// the HLL mean state; contact speed S_M = (rho v_d)_hll / rho_hll; star
// total pressure p* = rho_K (S_K - v_K)(S_M - v_K) + p_T,K (mean of both
// sides); on the side K of the face's region
//   rho* = rho_K (S_K - v_K)/(S_K - S_M), (rho v_d)* = rho* S_M,
//   (rho v_t)* = [rho_K v_t,K (S_K - v_K) - B_m (B_t,hll - B_t,K)]/(S_K - S_M),
//   B_t* = B_t,hll,
//   e* = [e_K (S_K - v_K) - p_T,K v_K + p* S_M + B_m (v_K.B_K - v_hll.B_hll)]/(S_K - S_M),
// and the flux F_K + S_K (U*_K - U_K), or F_L / F_R when the whole fan
// moves one way.
template <typename T>
__device__ __forceinline__ void hllc_sel(const T L0[NV], T pL0, const T R0[NV], T pR0, int d,
                                         T gamma, T gm1, T ch, T ch2, T f[NV])
{
    const T h = T(0.5);
    const int kB = BX + d;
    const T BdL = L0[kB], BdR = R0[kB];
    T Bm, psim;
    if (ch > T(0)) {
        Bm = h * (BdL + BdR) - Num<T>::div(R0[PSI] - L0[PSI], T(2) * ch);
        psim = h * (L0[PSI] + R0[PSI]) - h * ch * (BdR - BdL);
    } else {
        Bm = h * (BdL + BdR);
        psim = h * (L0[PSI] + R0[PSI]);
    }
    T U[2][NV], F[2][NV], v[2], pt[2], cf[2], vb[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const T *u0 = s ? R0 : L0;
        const T Bd0 = s ? BdR : BdL;
#pragma unroll
        for (int k = 0; k < NV; k++)
            U[s][k] = k == kB ? Bm : u0[k];
        Prim<T> w;
        w.ir = Num<T>::rcp(U[s][RHO]);
        w.vx = U[s][MX] * w.ir;
        w.vy = U[s][MY] * w.ir;
        w.vz = U[s][MZ] * w.ir;
        w.bb = U[s][BX] * U[s][BX] + U[s][BY] * U[s][BY] + U[s][BZ] * U[s][BZ];
        w.p = (s ? pR0 : pL0) + gm1 * (h * ((Bd0 - Bm) * (Bd0 + Bm)));
        flux_sel(U[s], w, d, ch2, F[s]);
        v[s] = d == 0 ? w.vx : (d == 1 ? w.vy : w.vz);
        pt[s] = w.p + h * w.bb;
        cf[s] = fast_sel(U[s], w, d, gamma);
        vb[s] = w.vx * U[s][BX] + w.vy * U[s][BY] + w.vz * U[s][BZ];
    }
    const T cmax = cf[0] > cf[1] ? cf[0] : cf[1];
    const T SL = (v[0] < v[1] ? v[0] : v[1]) - cmax;
    const T SR = (v[0] > v[1] ? v[0] : v[1]) + cmax;
    if (SL >= T(0) || SR <= T(0)) {
        const bool left = SL >= T(0);
#pragma unroll
        for (int k = 0; k < NV; k++)
            f[k] = left ? F[0][k] : F[1][k];
    } else {
        const T r = Num<T>::rcp(SR - SL);
        T hl[NV];
#pragma unroll
        for (int k = 0; k < EN; k++)
            hl[k] = (SR * U[1][k] - SL * U[0][k] - F[1][k] + F[0][k]) * r;
        hl[kB] = Bm;
        const T irh = Num<T>::rcp(hl[RHO]);
        const T vh[3] = {hl[MX] * irh, hl[MY] * irh, hl[MZ] * irh};
        const T SM = d == 0 ? vh[0] : (d == 1 ? vh[1] : vh[2]);
        const T vbh = vh[0] * hl[BX] + vh[1] * hl[BY] + vh[2] * hl[BZ];
        const T ps0 = U[0][RHO] * (SL - v[0]) * (SM - v[0]) + pt[0];
        const T ps1 = U[1][RHO] * (SR - v[1]) * (SM - v[1]) + pt[1];
        const T pst = h * (ps0 + ps1);
        const bool right = SM < T(0);
        const T S = right ? SR : SL;
        const T vs = right ? v[1] : v[0];
        const T pts = right ? pt[1] : pt[0];
        const T vbs = right ? vb[1] : vb[0];
        T us[NV], fs[NV];
#pragma unroll
        for (int k = 0; k < NV; k++) {
            us[k] = right ? U[1][k] : U[0][k];
            fs[k] = right ? F[1][k] : F[0][k];
        }
        const T sv = S - vs;
        const T iden = Num<T>::rcp(S - SM);
        T st[NV];
        st[RHO] = us[RHO] * sv * iden;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            st[MX + j] = j == d ? st[RHO] * SM
                                : (us[MX + j] * sv - Bm * (hl[BX + j] - us[BX + j])) * iden;
            st[BX + j] = j == d ? Bm : hl[BX + j];
        }
        st[EN] = (us[EN] * sv - pts * vs + pst * SM + Bm * (vbs - vbh)) * iden;
#pragma unroll
        for (int k = 0; k < EN + 1; k++)
            f[k] = fs[k] + S * (st[k] - us[k]);
    }
    f[kB] = psim;
    f[PSI] = ch2 * Bm;
}

// the face flux of the scheme's Riemann solver (RS = MAP_RUSANOV or MAP_HLLC)
template <int RS, int D, typename T>
__device__ __forceinline__ void face_flux(const T L[NV], T pL, const T R[NV], T pR, T gamma, T gm1,
                                          T ch, T ch2, T f[NV])
{
    if constexpr (RS == MAP_HLLC)
        hllc_sel(L, pL, R, pR, D, gamma, gm1, ch, ch2, f);
    else
        rusanov_sel(L, pL, R, pR, D, gamma, ch, ch2, f);
}

}  // namespace mapk
