// k_step_mmc3.hip -- the modified MacCormack block update (paper Sec. 3.1)
// on 3-D blocks, all directions together (Sec. 3.7): Lax-Friedrichs flux
// splitting f+- = (F_d(u) +- alpha u)/2 with the global alpha (c_h on the
// GLM pair B_d, psi), the predictor u~ = u - sum_d dt/dx_d (h_{i+1/2} -
// h_{i-1/2}) with h_{i+1/2} = f+_i + f-_{i+1}, and the limited corrector
// flux h_{i+1/2} + (Phi(g+_{i-1/2}, g+_{i+1/2}) - Phi(g-_{i+3/2}, g-_{i+1/2}))/2
// with g+_{i+1/2} = f~+_{i+1} - f+_i and g-_{i+1/2} = f-_{i+1} - f~-_i built
// from u~; then the EGLM sources and the resistive terms from u^n (Sec. 2,
// Sec. 3.5) and the exact psi damping.
//
// One block per workgroup of 4 waves, marching along z one plane per
// iteration.  Thread t owns the interior column (t % 16, t / 16); lanes 0-15
// of wave w also own the ring cell of side w (x = -1, x = 16, y = -1,
// y = 16) and lanes 16-35 the outer cells of the padded plane, as in the LF
// kernel.  Per plane p:
//   * u(p) is published to LDS; the in-plane split fluxes F_x(u), F_y(u) of
//     the whole padded plane are formed into one LDS buffer, one dimension
//     at a time, and give the x and y terms of u~(p) on the interior and
//     ring cells; the z term comes from the column's registers (the split
//     fluxes of planes p-1, p and p+1, each formed once) or, on ring cells,
//     from three ring planes kept in LDS;
//   * the z face p-1/2 is formed in the column's registers (each z face
//     once), which finishes plane p-1;
//   * on interior planes, F_x(u~), then F_y(u~), are formed on the cells
//     that the in-plane faces read, every in-plane face flux is formed once
//     into LDS, and each cell takes the difference of its two faces.
// A face flux is formed once and read by both of its cells, so a uniform
// state stays uniform bit for bit.  Ghost cells are read where the ghost
// descriptors point (Sec. 4.3), so U_out must not alias U_in.
#include <type_traits>

#include "kernels.hpp"
#include "physics.hpp"
#include "sched.hpp"
#include "tile.hpp"

namespace mapk {

namespace {
constexpr int NTM = NB * NB;          // threads: one per interior column
constexpr int XSM = PD * PD;          // padded plane (400)
constexpr int EW = NB + 2;            // E-plane edge (18)
constexpr int XE = EW * EW;           // E plane (324)
constexpr int NRM = 4 * NB;           // ring cells (no corners)
constexpr int NOM = 4 * PD;           // outer ring and ring corners
constexpr int OPWM = NOM / 4;         // outer cells per wave (20)
constexpr int NLDM = NRM + NOM;       // cells with a load role
constexpr int NFACE = (NB + 1) * NB;  // in-plane faces of one dimension (272)

__device__ __forceinline__ int pl(int x, int y) { return (y + NG) * PD + (x + NG); }
__device__ __forceinline__ int ei(int x, int y) { return (y + 1) * EW + (x + 1); }
}  // namespace

template <typename T, bool MIXED, bool RESIST, int LIM>
__global__ void __launch_bounds__(NTM) k_step_mmc3(StepArgs a)
{
    __shared__ T su[NV * XSM];           // u of plane p (padded plane)
    __shared__ T sF[NV * XSM];           // F_d(u(p)) of one dimension (padded plane)
    __shared__ T sut[NV * XE];           // u~(p) (E plane)
    __shared__ T sft[NV * XE];           // F_d(u~(p)) of one dimension (E plane)
    __shared__ T sfh[NV * NFACE];        // in-plane face fluxes of one dimension
    __shared__ T sring[3 * NV * NRM];    // ring cells of planes p-1, p, p+1
    __shared__ T sj[RESIST ? 5 * XSM : 1];  // eta J and eta (J x B) of plane p
    __shared__ size_t gld[5 * NLDM];     // load roles: source offsets per plane region

    const int t = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int ln = t & 63;
    const int qx = t % NB, qy = t / NB;
    const int q = pl(qx, qy);
    const bool isring = ln < NB;
    const bool isout = ln >= NB && ln < NB + OPWM;
    int li = 0, ex = 0, ey = 0;
    if (isring) {
        ex = wv == 0 ? -1 : (wv == 1 ? NB : ln);
        ey = wv == 2 ? -1 : (wv == 3 ? NB : ln);
        li = wv * NB + ln;
    } else if (isout) {
        const int c = wv * OPWM + ln - NB;
        if (c < PD) {
            ex = c - NG;
            ey = -NG;
        } else if (c < 2 * PD) {
            ex = c - PD - NG;
            ey = NB + 1;
        } else if (c < 2 * PD + NB + 2) {
            ex = -NG;
            ey = c - 2 * PD - 1;
        } else if (c < 2 * PD + 2 * (NB + 2)) {
            ex = NB + 1;
            ey = c - 2 * PD - (NB + 2) - 1;
        } else {
            const int cc = c - 2 * PD - 2 * (NB + 2);
            ex = (cc & 1) ? NB : -1;
            ey = (cc & 2) ? NB : -1;
        }
        li = NRM + c;
    }
    const int xq = pl(ex, ey);
    const int xe = isring ? ei(ex, ey) : 0;
    const int ri = wv * NB + ln;  // ring slot (ring lanes)

    Phys<T, MIXED> ph;
    ph.gamma = (T)a.gamma;
    ph.gm1 = (T)(a.gamma - 1.0);
    ph.gm1d = a.gamma - 1.0;
    const T *Uin = (const T *)a.Uin;
    T *Uout = (T *)a.Uout;
    T *fbuf = (T *)a.fbuf;
    constexpr int P3 = XSM * PD;
    constexpr int FC = NB * NB;

    int first, stride, end;
    xcd_range(a.nitems, first, stride, end);
    for (int item = first; item < end; item += stride) {
        const int slot = a.leaves[item];
        const BlockRec br = a.blk[slot];
        const map_dt rec = a.dt[br.sim];
        const double *dxp = a.lvl_dx + ((size_t)br.sim * (MAXL + 1) + br.level) * 3;
        T dtdx[3], i2d[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            dtdx[d] = (T)(rec.dt / dxp[d]);
            i2d[d] = (T)(0.5 / dxp[d]);
        }
        const T dt = (T)rec.dt, ch = (T)rec.ch, ch2 = (T)(rec.ch * rec.ch), damp = (T)rec.damp;
        const T alpha = (T)rec.alpha;
        const T eta = (T)a.eta;
        T *ob = Uout + (size_t)slot * NV * P3;

        // the split-flux speed of component v along D: c_h on the GLM pair
        auto al = [&](int v, int D) { return (v == BX + D || v == PSI) ? ch : alpha; };
        // u of the interior column at plane k (z ghost planes from the z
        // neighbours or the block's own prolongated ghosts)
        auto zbase = [&](int z) { return Uin + cell_src<3>(a.desc, slot, 0, 0, z) - (NG * PD + NG); };
        const T *const zb0 = zbase(-2), *const zb1 = zbase(-1), *const zb2 = zbase(0),
                      *const zb3 = zbase(NB), *const zb4 = zbase(NB + 1);
        auto load = [&](T(&dst)[NV], int k) {
            const T *p = (k == -2 ? zb0
                                  : (k == -1 ? zb1 : (k < NB ? zb2 + k * XSM : (k == NB ? zb3 : zb4)))) +
                         q;
#pragma unroll
            for (int v = 0; v < NV; v++)
                dst[v] = p[v * P3];
        };
        if (isring || isout) {
            const int zr[5] = {-2, -1, 0, NB, NB + 1};
#pragma unroll
            for (int r = 0; r < 5; r++)
                gld[r * NLDM + li] = cell_src<3>(a.desc, slot, ex, ey, zr[r]);
        }
        auto load_x = [&](T(&dst)[NV], int k) {
            const size_t o = k < 0 ? gld[(k + 2) * NLDM + li]
                                   : (k < NB ? gld[2 * NLDM + li] + (size_t)k * XSM
                                             : gld[(k - NB + 3) * NLDM + li]);
            const T *p = Uin + o;
#pragma unroll
            for (int v = 0; v < NV; v++)
                dst[v] = p[v * P3];
        };
        auto rslot = [&](int k) { return sring + ((k + 6) % 3) * (NV * NRM); };

        // split fluxes of a state along D
        auto split = [&](auto dc, const T u[NV], T (&fp)[NV], T (&fm)[NV]) {
            constexpr int D = decltype(dc)::value;
            T F[NV];
            ph.template flux<D, false>(u, ch2, F);
#pragma unroll
            for (int v = 0; v < NV; v++) {
                fp[v] = T(0.5) * (F[v] + al(v, D) * u[v]);
                fm[v] = T(0.5) * (F[v] - al(v, D) * u[v]);
            }
        };
        // F_D(u(p)) of the whole padded plane into sF
        auto plane_flux = [&](auto dc) {
            constexpr int D = decltype(dc)::value;
            for (int c = t; c < XSM; c += NTM) {
                T u[NV], F[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    u[v] = su[v * XSM + c];
                ph.template flux<D, false>(u, ch2, F);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    sF[v * XSM + c] = F[v];
            }
        };
        // f+ and f- of u(p) along D at padded index c (from sF and su)
        auto fpl = [&](int v, int c, int D) { return T(0.5) * (sF[v * XSM + c] + al(v, D) * su[v * XSM + c]); };
        auto fmi = [&](int v, int c, int D) { return T(0.5) * (sF[v * XSM + c] - al(v, D) * su[v * XSM + c]); };
        // the predictor term dt/dx_D (h_{c+1/2} - h_{c-1/2}) of the cell at c
        auto pred_term = [&](int v, int c, int s, int D) {
            const T hp = fpl(v, c, D) + fmi(v, c + s, D);
            const T hm = fpl(v, c - s, D) + fmi(v, c, D);
            return dtdx[D] * (hp - hm);
        };
        // F_D(u~(p)) of the cells the in-plane faces of D read (interior and
        // the ring sides across D) into sft
        auto tilde_flux = [&](auto dc) {
            constexpr int D = decltype(dc)::value;
            T u[NV], F[NV];
#pragma unroll
            for (int v = 0; v < NV; v++)
                u[v] = sut[v * XE + ei(qx, qy)];
            ph.template flux<D, false>(u, ch2, F);
#pragma unroll
            for (int v = 0; v < NV; v++)
                sft[v * XE + ei(qx, qy)] = F[v];
            if (isring && (wv >> 1) == D) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    u[v] = sut[v * XE + xe];
                ph.template flux<D, false>(u, ch2, F);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    sft[v * XE + xe] = F[v];
            }
        };
        // the limited flux of the in-plane face between the cells (x, y)
        // and (x, y) + e_D, with the block-face fluxes stored for reflux
        auto face = [&](auto dc, int x, int y, int k, int f) {
            constexpr int D = decltype(dc)::value;
            const int s = D == 0 ? 1 : PD, se = D == 0 ? 1 : EW;
            const int c = pl(x, y), e = ei(x, y);
            T fh[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const T a_ = al(v, D);
                const T *TF = sft + v * XE, *TU = sut + v * XE;
                const T tp0 = T(0.5) * (TF[e] + a_ * TU[e]);
                const T tp1 = T(0.5) * (TF[e + se] + a_ * TU[e + se]);
                const T tm0 = T(0.5) * (TF[e] - a_ * TU[e]);
                const T tm1 = T(0.5) * (TF[e + se] - a_ * TU[e + se]);
                const T h = fpl(v, c, D) + fmi(v, c + s, D);
                const T gp_m = tp0 - fpl(v, c - s, D);
                const T gp_p = tp1 - fpl(v, c, D);
                const T gm_p = fmi(v, c + s, D) - tm0;
                const T gm_pp = fmi(v, c + 2 * s, D) - tm1;
                fh[v] = h + T(0.5) * (limiter<LIM>(gp_m, gp_p) - limiter<LIM>(gm_pp, gm_p));
                sfh[v * NFACE + f] = fh[v];
            }
            const int cd = D == 0 ? x : y;
            const int side = cd == -1 ? 0 : (cd == NB - 1 ? 1 : -1);
            if (side >= 0) {
                const int fb = a.fbidx[(size_t)slot * 6 + 2 * D + side];
                if (fb >= 0) {
                    const int tt = (D == 0 ? y : x) + NB * k;
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        fbuf[((size_t)fb * NV + v) * FC + tt] = fh[v];
                }
            }
        };
        // eta J and eta (J x B) at padded index c, with the z neighbours' B
        auto curl = [&](int c, const T uc[NV], const T um_[NV], const T up_[NV], T (&e)[5], T &qz) {
            const T *bx = su + BX * XSM, *by = su + BY * XSM, *bz = su + BZ * XSM;
            const T dyBz = (bz[c + PD] - bz[c - PD]) * i2d[1];
            const T dzBy = (up_[BY] - um_[BY]) * i2d[2];
            const T dzBx = (up_[BX] - um_[BX]) * i2d[2];
            const T dxBz = (bz[c + 1] - bz[c - 1]) * i2d[0];
            const T dxBy = (by[c + 1] - by[c - 1]) * i2d[0];
            const T dyBx = (bx[c + PD] - bx[c - PD]) * i2d[1];
            const T jx = dyBz - dzBy, jy = dzBx - dxBz, jz = dxBy - dyBx;
            e[0] = eta * jx;
            e[1] = eta * jy;
            e[2] = eta * jz;
            e[3] = eta * (jz * uc[BY] - jy * uc[BZ]);
            e[4] = eta * (jx * uc[BZ] - jz * uc[BX]);
            qz = eta * (jy * uc[BX] - jx * uc[BY]);
        };

        // column registers: u of planes p-1 .. p+2, the z split fluxes
        // fp_z(p-1), fp_z(p), fm_z(p), the carried g+ of the face p-3/2 and
        // f~-_z(p-1), the z flux of the face p-3/2, the in-plane result of
        // plane p-1 (finished with its z faces), eta J of planes p-1, p-2
        T um[NV], u0[NV], up[NV], upp[NV];
        T fpz_m1[NV], fpz_0[NV], fmz_0[NV], gp_prev[NV], ftm_prev[NV], fz_prev[NV], Wc[NV];
        T jm1[3] = {T(0), T(0), T(0)}, jm2[3] = {T(0), T(0), T(0)};
        load(um, -2);
        load(u0, -1);
        load(up, 0);
        load(upp, 1);
        {
            T tmp[NV];
            split(std::integral_constant<int, 2>{}, um, fpz_m1, tmp);
            split(std::integral_constant<int, 2>{}, u0, fpz_0, fmz_0);
        }
#pragma unroll
        for (int v = 0; v < NV; v++) {
            gp_prev[v] = T(0);
            ftm_prev[v] = T(0);
            fz_prev[v] = T(0);
            Wc[v] = T(0);
        }
        T xr[NV], xc[NV];
        if (isring) {
            T r0[NV];
            load_x(r0, -1);
            T *rb = rslot(-1);
#pragma unroll
            for (int v = 0; v < NV; v++)
                rb[v * NRM + ri] = r0[v];
            load_x(xr, 0);
        } else if (isout) {
            load_x(xc, -1);
        }

        for (int p = -1; p <= NB; ++p) {
            const bool kI = p >= 0 && p < NB;
            // ---- (A) publish u(p); ring plane p+1; prefetch
#pragma unroll
            for (int v = 0; v < NV; v++)
                su[v * XSM + q] = u0[v];
            if (isring) {
                const T *rk = rslot(p);
                T *rn = rslot(p + 1);
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    su[v * XSM + xq] = rk[v * NRM + ri];
                    rn[v * NRM + ri] = xr[v];
                }
                if (p + 2 <= NB)
                    load_x(xr, p + 2);
            } else if (isout) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    su[v * XSM + xq] = xc[v];
                if (p + 1 <= NB)
                    load_x(xc, p + 1);
            }
            T un[NV];  // u(p+3), consumed two planes later
            if (p + 3 <= NB + 1) {
                load(un, p + 3);
            } else {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    un[v] = T(0);
            }
            __syncthreads();

            // ---- (B) F_x(u(p)); eta J of plane p
            plane_flux(std::integral_constant<int, 0>{});
            T jc[3] = {T(0), T(0), T(0)};
            if constexpr (RESIST) {
                T e[5], qz;
                curl(q, u0, um, up, e, qz);
#pragma unroll
                for (int i = 0; i < 5; i++)
                    sj[i * XSM + q] = e[i];
                jc[0] = e[0];
                jc[1] = e[1];
                jc[2] = qz;
                if (kI && isring) {
                    T ur[NV], urm[NV], urp[NV];
                    const T *rm = rslot(p - 1), *rp = rslot(p + 1);
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        ur[v] = su[v * XSM + xq];
                        urm[v] = rm[v * NRM + ri];
                        urp[v] = rp[v * NRM + ri];
                    }
                    T er[5], qr;
                    curl(xq, ur, urm, urp, er, qr);
#pragma unroll
                    for (int i = 0; i < 5; i++)
                        sj[i * XSM + xq] = er[i];
                }
            }
            __syncthreads();

            // ---- (C) x terms of u~(p)
            T acc[NV], accr[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                acc[v] = pred_term(v, q, 1, 0);
                accr[v] = T(0);
            }
            if (kI && isring) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    accr[v] = pred_term(v, xq, 1, 0);
            }
            __syncthreads();

            // ---- (D) F_y(u(p))
            plane_flux(std::integral_constant<int, 1>{});
            __syncthreads();

            // ---- (E) y and z terms, u~(p); the z face p-1/2 finishes plane p-1
            T fpz_p1[NV], fmz_p1[NV];
            split(std::integral_constant<int, 2>{}, up, fpz_p1, fmz_p1);
            T ut[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                acc[v] += pred_term(v, q, PD, 1);
                acc[v] += dtdx[2] * ((fpz_0[v] + fmz_p1[v]) - (fpz_m1[v] + fmz_0[v]));
                ut[v] = u0[v] - acc[v];
                sut[v * XE + ei(qx, qy)] = ut[v];
            }
            if (kI && isring) {
                T urm[NV], ur[NV], urp[NV];
                const T *rm = rslot(p - 1), *rp = rslot(p + 1);
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    urm[v] = rm[v * NRM + ri];
                    ur[v] = su[v * XSM + xq];
                    urp[v] = rp[v * NRM + ri];
                }
                T fpa[NV], fma[NV], fpb[NV], fmb[NV], fpc[NV], fmc[NV];
                split(std::integral_constant<int, 2>{}, urm, fpa, fma);
                split(std::integral_constant<int, 2>{}, ur, fpb, fmb);
                split(std::integral_constant<int, 2>{}, urp, fpc, fmc);
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    accr[v] += pred_term(v, xq, PD, 1);
                    accr[v] += dtdx[2] * ((fpb[v] + fmc[v]) - (fpa[v] + fmb[v]));
                    sut[v * XE + xe] = ur[v] - accr[v];
                }
            }
            {
                T ftp[NV], ftm[NV];
                split(std::integral_constant<int, 2>{}, ut, ftp, ftm);
                T fz[NV];
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const T gp_cur = ftp[v] - fpz_m1[v];
                    if (p >= 0) {
                        const T h = fpz_m1[v] + fmz_0[v];
                        const T gm_cur = fmz_0[v] - ftm_prev[v];
                        const T gm_nxt = fmz_p1[v] - ftm[v];
                        fz[v] = h + T(0.5) * (limiter<LIM>(gp_prev[v], gp_cur) -
                                              limiter<LIM>(gm_nxt, gm_cur));
                    } else {
                        fz[v] = T(0);
                    }
                    gp_prev[v] = gp_cur;
                    ftm_prev[v] = ftm[v];
                }
                if (p >= 1) {
                    T o[NV];
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        o[v] = Wc[v] - dtdx[2] * (fz[v] - fz_prev[v]);
                    if constexpr (RESIST) {
                        o[BX] = o[BX] + dt * ((jc[1] - jm2[1]) * i2d[2]);
                        o[BY] = o[BY] - dt * ((jc[0] - jm2[0]) * i2d[2]);
                        o[EN] = o[EN] + dt * ((jc[2] - jm2[2]) * i2d[2]);
                    }
                    o[PSI] = o[PSI] * damp;
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        ob[v * P3 + (p - 1 + NG) * XSM + q] = o[v];
                }
                if (p == 0 || p == NB) {
                    const int fb = a.fbidx[(size_t)slot * 6 + 4 + (p == NB ? 1 : 0)];
                    if (fb >= 0) {
                        const int tt = qx + NB * qy;
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            fbuf[((size_t)fb * NV + v) * FC + tt] = fz[v];
                    }
                }
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    fz_prev[v] = fz[v];
                    fpz_m1[v] = fpz_0[v];
                    fpz_0[v] = fpz_p1[v];
                    fmz_0[v] = fmz_p1[v];
                }
            }
            __syncthreads();

            if (kI) {
                // ---- (F, G) x faces: F_x(u~), F_x(u) again, then each face once
                tilde_flux(std::integral_constant<int, 0>{});
                plane_flux(std::integral_constant<int, 0>{});
                __syncthreads();
                for (int f = t; f < NFACE; f += NTM)
                    face(std::integral_constant<int, 0>{}, f % (NB + 1) - 1, f / (NB + 1), p, f);
                __syncthreads();
                T div[NV];
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const T *H = sfh + v * NFACE;
                    div[v] = dtdx[0] * (H[qy * (NB + 1) + qx + 1] - H[qy * (NB + 1) + qx]);
                }
                __syncthreads();
                // ---- (H, I) y faces
                tilde_flux(std::integral_constant<int, 1>{});
                plane_flux(std::integral_constant<int, 1>{});
                __syncthreads();
                for (int f = t; f < NFACE; f += NTM)
                    face(std::integral_constant<int, 1>{}, f % NB, f / NB - 1, p, f);
                __syncthreads();
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const T *H = sfh + v * NFACE;
                    div[v] += dtdx[1] * (H[(qy + 1) * NB + qx] - H[qy * NB + qx]);
                    Wc[v] = u0[v] - div[v];
                }
                // EGLM sources from central differences of u^n
                if (a.eglm) {
                    const T *bx = su + BX * XSM, *by = su + BY * XSM, *ps = su + PSI * XSM;
                    T divb = (bx[q + 1] - bx[q - 1]) * i2d[0];
                    T bgp = u0[BX] * ((ps[q + 1] - ps[q - 1]) * i2d[0]);
                    divb += (by[q + PD] - by[q - PD]) * i2d[1];
                    bgp += u0[BY] * ((ps[q + PD] - ps[q - PD]) * i2d[1]);
                    divb += (up[BZ] - um[BZ]) * i2d[2];
                    bgp += u0[BZ] * ((up[PSI] - um[PSI]) * i2d[2]);
                    Wc[MX] = Wc[MX] - dt * (divb * u0[BX]);
                    Wc[MY] = Wc[MY] - dt * (divb * u0[BY]);
                    Wc[MZ] = Wc[MZ] - dt * (divb * u0[BZ]);
                    Wc[EN] = Wc[EN] - dt * bgp;
                }
                // in-plane resistive terms -curl(eta J) and -div((eta J) x B)
                if constexpr (RESIST) {
                    const T *J0 = sj, *J1 = sj + XSM, *J2 = sj + 2 * XSM, *Q0 = sj + 3 * XSM,
                            *Q1 = sj + 4 * XSM;
                    Wc[BX] = Wc[BX] + dt * (-((J2[q + PD] - J2[q - PD]) * i2d[1]));
                    Wc[BY] = Wc[BY] + dt * ((J2[q + 1] - J2[q - 1]) * i2d[0]);
                    Wc[BZ] = Wc[BZ] + dt * ((J0[q + PD] - J0[q - PD]) * i2d[1] -
                                            (J1[q + 1] - J1[q - 1]) * i2d[0]);
                    Wc[EN] = Wc[EN] + dt * ((Q0[q + 1] - Q0[q - 1]) * i2d[0] +
                                            (Q1[q + PD] - Q1[q - PD]) * i2d[1]);
                }
            }
            __syncthreads();  // su, sF, sj reused by the next plane

            // ---- shift the column registers
#pragma unroll
            for (int v = 0; v < NV; v++) {
                um[v] = u0[v];
                u0[v] = up[v];
                up[v] = upp[v];
                upp[v] = un[v];
            }
#pragma unroll
            for (int i = 0; i < 3; i++) {
                jm2[i] = jm1[i];
                jm1[i] = jc[i];
            }
        }
    }
}

template <typename T, bool MIXED, bool RESIST>
static void launch_mmc3_lim(const StepArgs &a, int g, hipStream_t s)
{
    if (a.limiter == MAP_MINMOD)
        hipLaunchKernelGGL((k_step_mmc3<T, MIXED, RESIST, MAP_MINMOD>), dim3(g), dim3(NTM), 0, s, a);
    else if (a.limiter == MAP_VANLEER)
        hipLaunchKernelGGL((k_step_mmc3<T, MIXED, RESIST, MAP_VANLEER>), dim3(g), dim3(NTM), 0, s, a);
    else
        hipLaunchKernelGGL((k_step_mmc3<T, MIXED, RESIST, MAP_PAPER_PHI>), dim3(g), dim3(NTM), 0, s, a);
}

hipError_t launch_step_mmc3(bool fp64, bool resist, const StepArgs &a, int grid, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    const int g = grid > 0 ? (grid < a.nitems ? grid : a.nitems) : a.nitems;
    if (fp64) {
        if (resist)
            launch_mmc3_lim<double, false, true>(a, g, s);
        else
            launch_mmc3_lim<double, false, false>(a, g, s);
    } else {
        if (resist)
            launch_mmc3_lim<float, true, true>(a, g, s);
        else
            launch_mmc3_lim<float, true, false>(a, g, s);
    }
    return hipGetLastError();
}

}  // namespace mapk
