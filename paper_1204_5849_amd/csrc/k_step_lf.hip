// k_step_lf.hip -- the TVD-LF block update (paper Sec. 3.2, all directions
// together as in Sec. 3.7) with the EGLM source terms (Sec. 2), uniform
// resistivity (Sec. 3.5) and exact psi damping, for every leaf of a work list.
//
// Layout and schedule (gfx950): each workgroup owns whole blocks.  Threads own
// the columns of the block's padded cross-section (x in 2-D, x-y in 3-D) and
// march along the last axis (y in 2-D, z in 3-D), one plane per iteration:
//   * the march-axis neighbours of a cell (slopes, the half-step flux, the
//     face between planes, source and resistive differences) stay in
//     registers of the owning thread;
//   * in-plane neighbours are exchanged through LDS one plane at a time
//     (state, right face states, face fluxes, eta J), so LDS holds one plane
//     of a block instead of the whole padded tile (a 20^3 x 9 FP32 tile would
//     not fit in 160 KB);
//   * each face flux is evaluated once; the next plane is prefetched from
//     HBM while the current one is processed;
//   * ghost cells are read where the ghost descriptors point (Sec. 4.3): a
//     same-level neighbour's interior in U_in, with periodic wrap or outflow
//     clamping, or the block's own prolongated ghost region.  So no copy
//     pass fills same-level ghosts before the update, and U_out must not
//     alias U_in.
// 2-D workgroups hold 14 blocks, 3-D workgroups one block (5 waves).  A
// persistent grid strides over the work list.
#include <type_traits>

#include "kernels.hpp"
#include "physics.hpp"
#include "tile.hpp"

namespace mapk {

// Lane layout.  Only the columns whose face states feed a face compute: the
// ring one cell outside the interior, minus its corners in 3-D (which no
// face reads), i.e. 18 columns per 2-D block and 320 = 5 waves per 3-D block.
// The remaining cells of the padded plane (outer ring, 3-D ring corners)
// are only loaded, by the first threads, one plane ahead.
template <int NDIM>
struct SG;
template <>
struct SG<2> {
    static constexpr int XS = PD, BPW = 14, NT = 256, NCOL = NB + 2, NX = 2;
};
template <>
struct SG<3> {
    static constexpr int XS = PD * PD, BPW = 1, NT = 320, NCOL = 320, NX = 80;
};

// Rusanov flux (Equ:LFFlux) with alpha = max of the two fast speeds for the
// MHD components and c_h for the GLM pair (B_D, psi); the pressures of both
// states are given (computed once when the states were formed)
template <int D, typename T>
__device__ __forceinline__ void rusanov_p(const T L[NV], T pL, const T R[NV], T pR, T gamma,
                                          T ch, T ch2, T f[NV])
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
    flux_w<D>(L, wL, ch2, FL);
    flux_w<D>(R, wR, ch2, FR);
    const T sL = speed_w<D>(L, wL, gamma), sR = speed_w<D>(R, wR, gamma);
    const T al = sL > sR ? sL : sR;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        const T ak = (k == BX + D || k == PSI) ? ch : al;
        f[k] = T(0.5) * (FL[k] + FR[k]) - T(0.5) * ak * (R[k] - L[k]);
    }
}

template <int NDIM, typename T, bool MIXED, bool RESIST>
__global__ void __launch_bounds__(SG<NDIM>::NT) k_step_lf(StepArgs a)
{
    constexpr int XS = SG<NDIM>::XS, BPW = SG<NDIM>::BPW, DIN = NDIM - 1, MD = NDIM - 1;
    constexpr int P = XS * PD;
    constexpr int FC = NDIM == 3 ? NB * NB : NB;
    constexpr int SY = PD;  // in-plane y stride (3-D)
    __shared__ T su[BPW * NV * XS];
    __shared__ T srf[BPW * DIN * NV * XS];
    __shared__ T spr[BPW * DIN * XS];
    __shared__ T sj[RESIST ? BPW * 5 * XS : 1];
    // per thread: where its column (and its load-only cell) reads the plane
    // regions -2, -1, the interior (plane 0; plane k adds k XS), NB, NB+1
    constexpr int NXT = NDIM == 3 ? SG<3>::NX : SG<2>::NX * BPW;
    // (element offsets from Uin, so that the loads stay in the global
    // address space)
    __shared__ size_t gcol[5 * SG<NDIM>::NT];
    __shared__ size_t gxc[5 * NXT];

    // ---- this thread's column and its extra (load-only) cell
    const int t = threadIdx.x;
    int lb, qx, qy;
    bool lane;
    if constexpr (NDIM == 3) {
        lb = 0;
        lane = t < SG<3>::NCOL;
        if (t < NB) {
            qx = t;
            qy = -1;
        } else if (t < NB + NB * (NB + 2)) {
            const int r = t - NB;
            qy = r / (NB + 2);
            qx = r - qy * (NB + 2) - 1;
        } else {
            qx = t - NB - NB * (NB + 2);
            qy = NB;
        }
    } else {
        lb = t / SG<2>::NCOL;
        lane = lb < BPW;
        qx = t - lb * SG<2>::NCOL - 1;
        qy = 0;
    }
    if (!lane) {
        lb = 0;
        qx = 0;
        qy = 0;
    }
    const int q = (NDIM == 3 ? (qy + NG) * PD : 0) + qx + NG;
    int xq = -1, xlb = 0, ex = 0, ey = 0;
    if constexpr (NDIM == 3) {
        if (t < SG<3>::NX) {
            if (t < PD) {
                ex = t - NG;
                ey = -NG;
            } else if (t < 2 * PD) {
                ex = t - PD - NG;
                ey = NB + 1;
            } else if (t < 2 * PD + NB + 2) {
                ex = -NG;
                ey = t - 2 * PD - 1;
            } else if (t < 2 * PD + 2 * (NB + 2)) {
                ex = NB + 1;
                ey = t - 2 * PD - (NB + 2) - 1;
            } else {
                const int c = t - 2 * PD - 2 * (NB + 2);
                ex = (c & 1) ? NB : -1;
                ey = (c & 2) ? NB : -1;
            }
            xq = (ey + NG) * PD + ex + NG;
        }
    } else {
        if (t < SG<2>::NX * BPW) {
            xlb = t >> 1;
            xq = (t & 1) ? PD - 1 : 0;
            ex = xq - NG;
        }
    }
    const bool xI = qx >= 0 && qx < NB;
    const bool yI = NDIM == 2 || (qy >= 0 && qy < NB);
    const bool inI = lane && xI && yI;

    Phys<T, MIXED> ph;
    ph.gamma = (T)a.gamma;
    ph.gm1 = (T)(a.gamma - 1.0);
    ph.gm1d = a.gamma - 1.0;
    const T gam = (T)a.gamma;
    const T *Uin = (const T *)a.Uin;
    T *Uout = (T *)a.Uout;
    T *fbuf = (T *)a.fbuf;
    const int lim = a.limiter;

    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        // 3-D: one block per workgroup, so the block and everything derived
        // from it are wave-uniform (scalar registers)
        const int li = NDIM == 3 ? item : item * BPW + lb;
        const bool has = NDIM == 3 ? (item < a.nleaves) : (lane && li < a.nleaves);
        const int slot = NDIM == 3 ? a.leaves[item] : (has ? a.leaves[li] : 0);
        const int lix = item * BPW + xlb;
        const bool xhas = xq >= 0 && lix < a.nleaves;
        const int xslot = xhas ? a.leaves[lix] : 0;
        const BlockRec br = a.blk[slot];
        const map_dt rec = a.dt[br.sim];
        const double *dxp = a.lvl_dx + ((size_t)br.sim * (MAXL + 1) + br.level) * 3;
        T dtdx[NDIM], hdt[NDIM], i2d[NDIM];
#pragma unroll
        for (int d = 0; d < NDIM; d++) {
            double r = rec.dt / dxp[d];
            dtdx[d] = (T)r;
            hdt[d] = (T)(0.5 * r);
            i2d[d] = (T)(0.5 / dxp[d]);
        }
        const T dt = (T)rec.dt, ch = (T)rec.ch, ch2 = (T)(rec.ch * rec.ch), damp = (T)rec.damp;
        const T eta = (T)a.eta;
        T *ob = Uout + (size_t)slot * NV * P;

        auto set_src = [&](size_t *tab, int stride, int sl, int cx, int cy) {
            const int zr[5] = {-2, -1, 0, NB, NB + 1};
#pragma unroll
            for (int r = 0; r < 5; r++) {
                if constexpr (NDIM == 3)
                    tab[r * stride] = cell_src<3>(a.desc, sl, cx, cy, zr[r]);
                else
                    tab[r * stride] = cell_src<2>(a.desc, sl, cx, zr[r], 0);
            }
        };
        // k is the same for the whole workgroup: the region choice is uniform
        auto src_of = [&](const size_t *tab, int stride, int k) -> const T * {
            if (k < 0)
                return Uin + tab[(k + 2) * stride];
            if (k < NB)
                return Uin + tab[2 * stride] + k * XS;
            return Uin + tab[(k - NB + 3) * stride];
        };
        if (has)
            set_src(gcol + t, SG<NDIM>::NT, slot, qx, qy);
        if (xhas)
            set_src(gxc + t, NXT, xslot, ex, ey);

        auto load = [&](T(&dst)[NV], int k) {
            if (has) {
                const T *p = src_of(gcol + t, SG<NDIM>::NT, k);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    dst[v] = p[v * P];
            } else {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    dst[v] = T(0);
                dst[RHO] = T(1);
                dst[EN] = T(4);
            }
        };
        auto load_x = [&](T(&dst)[NV], int k) {
            if (xhas) {
                const T *p = src_of(gxc + t, NXT, k);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    dst[v] = p[v * P];
            }
        };

        T um[NV], u0[NV], up[NV], upp[NV], xc[NV];
        load(um, -2);
        load(u0, -1);
        load(up, 0);
        load_x(xc, -1);
        // carried to the next plane: Wc = u - (in-plane flux differences)
        // + dt (sources + in-plane resistive terms), the flux of the face
        // k-1/2 (the march-axis difference is taken as a difference, so a
        // uniform state stays exactly uniform), the left state of the face
        // k+1/2, and eta J of the two previous planes
        T Lm_prev[NV], Wc[NV], fm_prev[NV];
        T pLm_prev = T(1);
        T jm1[3], jm2[3];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            Lm_prev[v] = T(0);
            Wc[v] = T(0);
            fm_prev[v] = T(0);
        }
#pragma unroll
        for (int i = 0; i < 3; i++) {
            jm1[i] = T(0);
            jm2[i] = T(0);
        }

        for (int k = -1; k <= NB; ++k) {
            const bool kI = k >= 0 && k < NB;
            // ---- (A) publish plane k (own column and the load-only cell)
            if (lane) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    su[(lb * NV + v) * XS + q] = u0[v];
            }
            if (xhas) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    su[(xlb * NV + v) * XS + xq] = xc[v];
            }
            if (k + 2 <= NB + 1)
                load(upp, k + 2);
            if (k + 1 <= NB + 1)
                load_x(xc, k + 1);
            __syncthreads();

            T Lin[DIN][NV], pLin[DIN], Lm[NV], Rm[NV];
            T pLm = T(1), pRm = T(1);
            T src[4] = {T(0), T(0), T(0), T(0)};
            T jc[3] = {T(0), T(0), T(0)};
            // planes -1 and NB only feed the faces between planes: interior columns
            const bool work = lane && (kI || inI);
            if (work) {
                // slopes from the old-time differences (limiter1)
                T dl[NDIM][NV];
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const T *row = su + (lb * NV + v) * XS;
                    dl[0][v] = limiter(lim, u0[v] - row[q - 1], row[q + 1] - u0[v]);
                    if constexpr (NDIM == 3)
                        dl[1][v] = limiter(lim, u0[v] - row[q - SY], row[q + SY] - u0[v]);
                    dl[MD][v] = limiter(lim, u0[v] - um[v], up[v] - u0[v]);
                }
                // half-step predictor u~ = u - dt/(2dx) sum_d [f(u + D/2) - f(u - D/2)],
                // evaluated optimistically; if any face state of the cell has
                // rho <= 0 or p <= 0 the slopes fall back to zero and u~ = u
                T acc[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    acc[v] = T(0);
                bool ok = true;
                auto pred = [&](auto dc) {
                    constexpr int d = decltype(dc)::value;
                    T s1[NV], f1[NV], f2[NV];
                    Prim<T> w;
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        s1[v] = u0[v] + T(0.5) * dl[d][v];
                    prim_of(ph, s1, w);
                    ok = ok && admissible_w(s1, w);
                    flux_w<d>(s1, w, ch2, f1);
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        s1[v] = u0[v] - T(0.5) * dl[d][v];
                    prim_of(ph, s1, w);
                    ok = ok && admissible_w(s1, w);
                    flux_w<d>(s1, w, ch2, f2);
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        acc[v] += hdt[d] * (f1[v] - f2[v]);
                };
                pred(std::integral_constant<int, 0>{});
                pred(std::integral_constant<int, 1>{});
                if constexpr (NDIM == 3)
                    pred(std::integral_constant<int, 2>{});
                if (!ok) {
#pragma unroll
                    for (int d = 0; d < NDIM; d++)
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            dl[d][v] = T(0);
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        acc[v] = T(0);
                    if (has)
                        atomicAdd(&a.cnt[0], 1ull);
                }
                T ut[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    ut[v] = u0[v] - acc[v];
                // face states with the old-time slopes (limiter2); a state with
                // rho <= 0 or p <= 0 is replaced by the cell's u~
                const int qc[3] = {qx, NDIM == 3 ? qy : k, k};
#pragma unroll
                for (int d = 0; d < NDIM; d++) {
                    T L[NV], R[NV];
                    Prim<T> wl, wr;
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        L[v] = ut[v] + T(0.5) * dl[d][v];
                        R[v] = ut[v] - T(0.5) * dl[d][v];
                    }
                    prim_of(ph, L, wl);
                    prim_of(ph, R, wr);
                    bool others = true;
#pragma unroll
                    for (int e = 0; e < NDIM; e++)
                        if (e != d)
                            others = others && qc[e] >= 0 && qc[e] < NB;
                    if (!admissible_w(L, wl)) {
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            L[v] = ut[v];
                        prim_of(ph, L, wl);
                        if (has && others && qc[d] < NB)
                            atomicAdd(&a.cnt[1], 1ull);
                    }
                    if (!admissible_w(R, wr)) {
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            R[v] = ut[v];
                        prim_of(ph, R, wr);
                        if (has && others && qc[d] >= 0)
                            atomicAdd(&a.cnt[1], 1ull);
                    }
                    if (d < DIN) {
#pragma unroll
                        for (int v = 0; v < NV; v++) {
                            srf[((lb * DIN + d) * NV + v) * XS + q] = R[v];
                            Lin[d < DIN ? d : 0][v] = L[v];
                        }
                        spr[(lb * DIN + d) * XS + q] = wr.p;
                        pLin[d < DIN ? d : 0] = wl.p;
                    } else {
#pragma unroll
                        for (int v = 0; v < NV; v++) {
                            Lm[v] = L[v];
                            Rm[v] = R[v];
                        }
                        pLm = wl.p;
                        pRm = wr.p;
                    }
                }
                // EGLM sources from central differences of u^n
                if (a.eglm && inI && kI) {
                    const T *bx = su + (lb * NV + BX) * XS, *by = su + (lb * NV + BY) * XS;
                    const T *ps = su + (lb * NV + PSI) * XS;
                    T divb = (bx[q + 1] - bx[q - 1]) * i2d[0];
                    T bgp = u0[BX] * ((ps[q + 1] - ps[q - 1]) * i2d[0]);
                    if constexpr (NDIM == 3) {
                        divb += (by[q + SY] - by[q - SY]) * i2d[1];
                        bgp += u0[BY] * ((ps[q + SY] - ps[q - SY]) * i2d[1]);
                    }
                    divb += (up[BX + MD] - um[BX + MD]) * i2d[MD];
                    bgp += u0[BX + MD] * ((up[PSI] - um[PSI]) * i2d[MD]);
                    src[0] = divb * u0[BX];
                    src[1] = divb * u0[BY];
                    src[2] = divb * u0[BZ];
                    src[3] = bgp;
                }
                // resistivity: eta J and eta (J x B) on this plane
                if constexpr (RESIST) {
                    const T *bx = su + (lb * NV + BX) * XS, *by = su + (lb * NV + BY) * XS;
                    const T *bz = su + (lb * NV + BZ) * XS;
                    T jx, jy, jz;
                    if constexpr (NDIM == 3) {
                        T dyBz = (bz[q + SY] - bz[q - SY]) * i2d[1];
                        T dzBy = (up[BY] - um[BY]) * i2d[2];
                        T dzBx = (up[BX] - um[BX]) * i2d[2];
                        T dxBz = (bz[q + 1] - bz[q - 1]) * i2d[0];
                        T dxBy = (by[q + 1] - by[q - 1]) * i2d[0];
                        T dyBx = (bx[q + SY] - bx[q - SY]) * i2d[1];
                        jx = dyBz - dzBy;
                        jy = dzBx - dxBz;
                        jz = dxBy - dyBx;
                    } else {
                        T dyBz = (up[BZ] - um[BZ]) * i2d[1];
                        T dxBz = (bz[q + 1] - bz[q - 1]) * i2d[0];
                        T dxBy = (by[q + 1] - by[q - 1]) * i2d[0];
                        T dyBx = (up[BX] - um[BX]) * i2d[1];
                        jx = dyBz;
                        jy = -dxBz;
                        jz = dxBy - dyBx;
                    }
                    T ejx = eta * jx, ejy = eta * jy, ejz = eta * jz;
                    T qx_ = eta * (jz * u0[BY] - jy * u0[BZ]);
                    T qy_ = eta * (jx * u0[BZ] - jz * u0[BX]);
                    T qz_ = eta * (jy * u0[BX] - jx * u0[BY]);
                    T *J = sj + lb * 5 * XS;
                    J[0 * XS + q] = ejx;
                    J[1 * XS + q] = ejy;
                    J[2 * XS + q] = ejz;
                    J[3 * XS + q] = qx_;
                    J[4 * XS + q] = qy_;
                    if constexpr (NDIM == 3) {
                        jc[0] = ejx;
                        jc[1] = ejy;
                        jc[2] = qz_;
                    } else {
                        jc[0] = ejx;
                        jc[1] = ejz;
                        jc[2] = qy_;
                    }
                }
            }
            __syncthreads();  // (B) right face states, their pressures and eta J published

            // ---- fluxes of the in-plane faces of plane k and of the face k-1/2
            T fin[DIN][NV];
            bool dof[DIN];
            T rin[4] = {T(0), T(0), T(0), T(0)};
            dof[0] = kI && lane && qx >= -1 && qx < NB && yI;
            if constexpr (NDIM == 3)
                dof[DIN - 1] = kI && lane && qy >= -1 && qy < NB && xI;
            if (dof[0]) {
                T R[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    R[v] = srf[((lb * DIN + 0) * NV + v) * XS + q + 1];
                rusanov_p<0>(Lin[0], pLin[0], R, spr[(lb * DIN + 0) * XS + q + 1], gam, ch, ch2,
                             fin[0]);
            }
            if constexpr (NDIM == 3) {
                if (dof[1]) {
                    T R[NV];
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        R[v] = srf[((lb * DIN + 1) * NV + v) * XS + q + SY];
                    rusanov_p<1>(Lin[1], pLin[1], R, spr[(lb * DIN + 1) * XS + q + SY], gam, ch,
                                 ch2, fin[1]);
                }
            }
            if constexpr (RESIST) {
                if (inI && kI) {
                    const T *J = sj + lb * 5 * XS;
                    const T *J0 = J, *J1 = J + XS, *J2 = J + 2 * XS, *Q0 = J + 3 * XS, *Q1 = J + 4 * XS;
                    if constexpr (NDIM == 3) {
                        rin[0] = -((J2[q + SY] - J2[q - SY]) * i2d[1]);
                        rin[1] = (J2[q + 1] - J2[q - 1]) * i2d[0];
                        rin[2] = (J0[q + SY] - J0[q - SY]) * i2d[1] - (J1[q + 1] - J1[q - 1]) * i2d[0];
                        rin[3] = (Q0[q + 1] - Q0[q - 1]) * i2d[0] + (Q1[q + SY] - Q1[q - SY]) * i2d[1];
                    } else {
                        rin[0] = (J2[q + 1] - J2[q - 1]) * i2d[0];
                        rin[1] = (J1[q + 1] - J1[q - 1]) * i2d[0];
                        rin[2] = (Q0[q + 1] - Q0[q - 1]) * i2d[0];
                    }
                }
            }
            const bool dom = inI && k >= 0;
            T fmc[NV];
            if (dom)
                rusanov_p<MD>(Lm_prev, pLm_prev, Rm, pRm, gam, ch, ch2, fmc);
            __syncthreads();  // (C) all reads of the right face states done
#pragma unroll
            for (int d = 0; d < DIN; d++)
                if (dof[d]) {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        srf[((lb * DIN + d) * NV + v) * XS + q] = fin[d][v];
                }
            // fluxes of block faces shared with another level (reflux)
            if (has) {
#pragma unroll
                for (int d = 0; d < DIN; d++) {
                    if (!dof[d])
                        continue;
                    const int qd = d == 0 ? qx : qy;
                    const int side = qd == -1 ? 0 : (qd == NB - 1 ? 1 : -1);
                    if (side < 0)
                        continue;
                    const int fb = a.fbidx[(size_t)slot * 6 + 2 * d + side];
                    if (fb < 0)
                        continue;
                    int tt;
                    if constexpr (NDIM == 3)
                        tt = (d == 0 ? qy : qx) + NB * k;
                    else
                        tt = k;
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        fbuf[((size_t)fb * NV + v) * FC + tt] = fin[d][v];
                }
                if (dom && (k == 0 || k == NB)) {
                    const int fb = a.fbidx[(size_t)slot * 6 + 2 * MD + (k == NB ? 1 : 0)];
                    if (fb >= 0) {
                        const int tt = NDIM == 3 ? qx + NB * qy : qx;
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            fbuf[((size_t)fb * NV + v) * FC + tt] = fmc[v];
                    }
                }
            }
            __syncthreads();  // (D) in-plane face fluxes published

            // ---- finalise plane k-1 with the face k-1/2: march-axis flux
            //      difference, march-axis resistive terms, psi damping (MHD-5
            //      integrated exactly)
            if (dom && k >= 1 && has) {
                T o[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    o[v] = Wc[v] - dtdx[MD] * (fmc[v] - fm_prev[v]);
                if constexpr (RESIST) {
                    if constexpr (NDIM == 3) {
                        o[BX] = o[BX] + dt * ((jc[1] - jm2[1]) * i2d[2]);
                        o[BY] = o[BY] - dt * ((jc[0] - jm2[0]) * i2d[2]);
                        o[EN] = o[EN] + dt * ((jc[2] - jm2[2]) * i2d[2]);
                    } else {
                        o[BX] = o[BX] - dt * ((jc[1] - jm2[1]) * i2d[1]);
                        o[BZ] = o[BZ] + dt * ((jc[0] - jm2[0]) * i2d[1]);
                        o[EN] = o[EN] + dt * ((jc[2] - jm2[2]) * i2d[1]);
                    }
                }
                o[PSI] = o[PSI] * damp;
#pragma unroll
                for (int v = 0; v < NV; v++)
                    ob[v * P + (k - 1 + NG) * XS + q] = o[v];
            }
            // ---- start plane k: in-plane flux differences, EGLM sources and
            //      in-plane resistive terms
            if (inI && kI) {
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    T acc = dtdx[0] * (fin[0][v] - srf[((lb * DIN + 0) * NV + v) * XS + q - 1]);
                    if constexpr (NDIM == 3)
                        acc += dtdx[1] * (fin[1][v] - srf[((lb * DIN + 1) * NV + v) * XS + q - SY]);
                    Wc[v] = u0[v] - acc;
                }
                if (a.eglm) {
                    Wc[MX] = Wc[MX] - dt * src[0];
                    Wc[MY] = Wc[MY] - dt * src[1];
                    Wc[MZ] = Wc[MZ] - dt * src[2];
                    Wc[EN] = Wc[EN] - dt * src[3];
                }
                if constexpr (RESIST) {
                    if constexpr (NDIM == 3) {
                        Wc[BX] = Wc[BX] + dt * rin[0];
                        Wc[BY] = Wc[BY] + dt * rin[1];
                        Wc[BZ] = Wc[BZ] + dt * rin[2];
                        Wc[EN] = Wc[EN] + dt * rin[3];
                    } else {
                        Wc[BY] = Wc[BY] + dt * rin[0];
                        Wc[BZ] = Wc[BZ] - dt * rin[1];
                        Wc[EN] = Wc[EN] + dt * rin[2];
                    }
                }
            }
            // ---- shift the march-axis registers
#pragma unroll
            for (int v = 0; v < NV; v++) {
                fm_prev[v] = dom ? fmc[v] : T(0);
                Lm_prev[v] = work ? Lm[v] : T(0);
                um[v] = u0[v];
                u0[v] = up[v];
                up[v] = upp[v];
            }
            pLm_prev = pLm;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                jm2[i] = jm1[i];
                jm1[i] = jc[i];
            }
        }
        __syncthreads();  // LDS reuse by the next work item
    }
}

template <int NDIM, typename T, bool MIXED, bool RESIST>
static hipError_t launch_one(const StepArgs &a, int grid, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    int g = grid > 0 ? (grid < a.nitems ? grid : a.nitems) : a.nitems;
    hipLaunchKernelGGL((k_step_lf<NDIM, T, MIXED, RESIST>), dim3(g), dim3(SG<NDIM>::NT), 0, s, a);
    return hipGetLastError();
}

int step_blocks_per_group(int ndim, int scheme)
{
    if (scheme == MAP_MMC)
        return 1;
    return ndim == 3 ? SG<3>::BPW : SG<2>::BPW;
}

hipError_t launch_step_lf(int ndim, bool fp64, bool resist, const StepArgs &a, int grid,
                          hipStream_t s)
{
    if (ndim == 2) {
        if (fp64)
            return resist ? launch_one<2, double, false, true>(a, grid, s)
                          : launch_one<2, double, false, false>(a, grid, s);
        return resist ? launch_one<2, float, true, true>(a, grid, s)
                      : launch_one<2, float, true, false>(a, grid, s);
    }
    if (fp64)
        return resist ? launch_one<3, double, false, true>(a, grid, s)
                      : launch_one<3, double, false, false>(a, grid, s);
    return resist ? launch_one<3, float, true, true>(a, grid, s)
                  : launch_one<3, float, true, false>(a, grid, s);
}

}  // namespace mapk
