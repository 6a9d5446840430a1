// k_step3.hpp -- the block update of 3-D leaf blocks: the TVD-LF step
// (paper Sec. 3.2) or one stage of WENO with TVD Runge-Kutta 2 (Sec. 3.3),
// all directions together (Sec. 3.7), with the EGLM source terms (Sec. 2),
// uniform resistivity (Sec. 3.5) and exact psi damping.
//
// Schedule (gfx950): one block per workgroup of 4 waves, so that two
// workgroups share a compute unit (the FP32 kernel keeps to 256 registers
// and 80 KB of LDS per workgroup) and one block's waits overlap the other's
// arithmetic; an FP32 instance compiled for one workgroup per CU (512
// registers, no spills) is the launch autotuner's alternative.  Threads own the 16 x 16 interior columns of the block and
// march along z one plane per iteration:
//   * march-axis neighbours (slopes, the half-step flux, the face between
//     planes, source and resistive differences) stay in the thread's
//     registers; in-plane neighbours are exchanged through LDS one plane at
//     a time (state, right face states, face fluxes, eta J).  LF takes two
//     barriers per plane, face states published and face fluxes published,
//     and writes the state of plane k+1 between the two into the slot of
//     plane k-1, which has no reader left after the first; the WENO stages
//     publish plane k behind a third barrier at the top of its iteration;
//   * the ring of cells just outside the interior (minus its corners) feeds
//     the block's boundary faces: lanes 0-15 of wave w own the ring side w
//     (x = -1, x = 16, y = -1, y = 16) and load its cells two planes ahead
//     through a small LDS buffer; the reduced pass over a plane's 64 ring
//     cells (for LF the predictor, then the one face state the interior
//     reads) runs on one wave, one lane per cell, the wave taking turns
//     with the plane index, so that the other three waves issue nothing for
//     it (for WENO, whose pass is a few face states, on the ring lanes of
//     every wave); lanes 0-15 of the waves of the -1 sides form the flux of
//     that face;
//   * lanes 16-35 of each wave load the remaining cells of the padded plane
//     (outer ring and ring corners), one plane ahead;
//   * interior columns read their planes from the block itself or, for the
//     ghost planes, from the z-neighbours' interiors (wave-uniform bases);
//     ring and outer cells read where their ghost descriptors point (Sec.
//     4.3), so U_out must not alias U_in;
//   * each face flux is evaluated once and the march-axis flux difference is
//     formed explicitly, so a uniform state stays exactly uniform;
//   * WENO stages differ only in the face states (three-cell WENO along
//     each dimension, no predictor) and in the end of the update: stage 1
//     stores u1 without damping, stage 2 stores (u + u1 + dt L(u1)) / 2, u
//     read from U_base at the cell itself, then damps psi, and the reflux
//     face fluxes become the mean of both stages' fluxes.
// A persistent grid strides over the leaf list.  The FP32 resistive LF and
// first WENO stage instances are compiled in k_step3_ilp.hip, the others in
// k_step3.hip: they take different instruction schedulers (see the build
// script).
#pragma once

#include <type_traits>

#include "kernels.hpp"
#include "physics.hpp"
#include "step_common.hpp"
#include "sched.hpp"
#include "tile.hpp"

namespace mapk {

namespace {
constexpr int NT3 = NB * NB;          // threads: one per interior column
constexpr int XS3 = PD * PD;          // plane stride
constexpr int P3 = XS3 * PD;          // padded tile cells
constexpr int NRING = 4 * NB;         // ring cells of a plane (one side per wave)
constexpr int NOUT = 4 * PD + 4;      // outer-ring cells and ring corners (load only)
constexpr int NLD = NRING + NOUT;     // cells loaded by the load lanes
constexpr int OPW = NOUT / 4;         // outer cells per wave (20)
static_assert(NB == 16 && NT3 == 256, "lane layout assumes 16^3 blocks");
}  // namespace

template <typename T, bool MIXED, bool RESIST, int SCH, int LIM, int RS, int OCC>
__global__ void __launch_bounds__(NT3, OCC) k_step3(StepArgs a)
{
    constexpr int SY = PD;
    constexpr int SUB = NV * XS3;
    __shared__ T su[2 * SUB];               // state of planes k and k-1 (by parity)
    __shared__ T srf[2 * NV * XS3];         // in-plane right face states, then fluxes
    __shared__ T spr[2 * XS3];              // pressures of those face states
    __shared__ T sj[RESIST ? 5 * XS3 : 1];  // eta J and eta (J x B) of plane k
    __shared__ T sring[2 * NV * NRING];     // ring cells of planes k and k+1 (by parity)
    __shared__ size_t gld[5 * NLD];         // load lanes: source offsets per plane region

    const int t = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // wave (uniform)
    const int ln = t & 63;
    // interior column of this thread
    const int qx = t % NB, qy = t / NB;
    const int q = (qy + NG) * PD + qx + NG;
    // load role: ring cell (lanes 0-15, side = wave) or outer cell (16-35)
    const bool isring = ln < NB;
    const bool isout = ln >= NB && ln < NB + OPW;
    int li = 0, ex = 0, ey = 0;
    if (isring) {
        ex = wv == 0 ? -1 : (wv == 1 ? NB : ln);
        ey = wv == 2 ? -1 : (wv == 3 ? NB : ln);
        li = wv * NB + ln;
    } else if (isout) {
        const int c = wv * OPW + ln - NB;
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
        li = NRING + c;
    }
    const int xq = (ey + NG) * PD + ex + NG;
    const int ri = wv * NB + ln;  // ring slot (isring lanes)
    // the ring side of this wave: dimension of the face it feeds and whether
    // the ring cell is the left state of the face -1/2 (x or y = -1)
    const int rdim = wv >> 1;
    const bool rlo = (wv & 1) == 0;
    // ring-pass role.  LF: every lane of the wave that runs the ring pass of
    // a plane, ring cell ln on side ln / 16.  WENO (whose ring pass is a few
    // face states, cheaper than moving it): the ring lanes of every wave
    constexpr bool RING1 = SCH == SCH_LF;
    // LF: two barriers per plane, the next plane published between them;
    // WENO stages: a third barrier after publishing plane k at the top of
    // its iteration (the WENO stages measured no faster, with HLLC slower,
    // in the two-barrier form)
    constexpr bool TWOB = SCH == SCH_LF;
    const int rsd = ln >> 4, rix = ln & 15;
    const int rex = rsd == 0 ? -1 : (rsd == 1 ? NB : rix);
    const int rey = rsd == 2 ? -1 : (rsd == 3 ? NB : rix);
    const int xqr = RING1 ? (rey + NG) * PD + rex + NG : xq;
    const int rir = RING1 ? ln : ri;
    const int rdr = RING1 ? rsd >> 1 : rdim;
    const bool rlr = RING1 ? (rsd & 1) == 0 : rlo;

    Phys<T, MIXED> ph;
    ph.gamma = (T)a.gamma;
    ph.gm1 = (T)(a.gamma - 1.0);
    ph.gm1d = a.gamma - 1.0;
    const T gam = (T)a.gamma;
    const T *Uin = (const T *)a.Uin;
    T *Uout = (T *)a.Uout;
    T *fbuf = (T *)a.fbuf;
    constexpr int FC = NB * NB;
    // a reflux face flux: the step's own, or for the second WENO stage the
    // mean with the first stage's
    auto put_flux = [&](size_t i, T f) {
        if constexpr (SCH == SCH_WENO2)
            fbuf[i] = T(0.5) * fbuf[i] + T(0.5) * f;
        else
            fbuf[i] = f;
    };

    // neighbouring blocks on one XCD, so that the ghost cells read from
    // neighbours come from that XCD's L2
    int first, stride, end;
    xcd_range(a.nitems, first, stride, end);
    for (int item = first; item < end; item += stride) {
        const int slot = a.leaves[item];
        const BlockRec br = a.blk[slot];
        const map_dt rec = a.dt[br.sim];
        const double *dxp = a.lvl_dx + ((size_t)br.sim * (MAXL + 1) + br.level) * 3;
        T dtdx[3], hdt[3], i2d[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const double r = rec.dt / dxp[d];
            dtdx[d] = (T)r;
            hdt[d] = (T)(0.5 * r);
            i2d[d] = (T)(0.5 / dxp[d]);
        }
        const T dt = (T)rec.dt, ch = (T)rec.ch, ch2 = (T)(rec.ch * rec.ch), damp = (T)rec.damp;
        const T eta = (T)a.eta;
        T *ob = Uout + (size_t)slot * NV * P3;

        // interior columns: planes -2, -1 and NB, NB+1 come from the z
        // neighbours (or the block's own prolongated / clamped ghosts), the
        // interior planes from the block; the bases are the same for every
        // thread
        // (base + q addresses the column's cell of the plane)
        auto zbase = [&](int z) { return Uin + cell_src<3>(a.desc, slot, 0, 0, z) - (NG * PD + NG); };
        const T *const zb0 = zbase(-2), *const zb1 = zbase(-1), *const zb2 = zbase(0),
                      *const zb3 = zbase(NB), *const zb4 = zbase(NB + 1);
        auto load = [&](T(&dst)[NV], int k) {
            const T *p = (k == -2 ? zb0
                                  : (k == -1 ? zb1 : (k < NB ? zb2 + k * XS3 : (k == NB ? zb3 : zb4)))) +
                         q;
#pragma unroll
            for (int v = 0; v < NV; v++)
                dst[v] = p[v * P3];
        };
        // load lanes: per-cell sources of the five plane regions
        const bool isld = isring || isout;
        if (isld) {
            const int zr[5] = {-2, -1, 0, NB, NB + 1};
#pragma unroll
            for (int r = 0; r < 5; r++)
                gld[r * NLD + li] = cell_src<3>(a.desc, slot, ex, ey, zr[r]);
        }
        auto load_x = [&](T(&dst)[NV], int k) {
            const size_t o = k < 0 ? gld[(k + 2) * NLD + li]
                                   : (k < NB ? gld[2 * NLD + li] + (size_t)k * XS3
                                             : gld[(k - NB + 3) * NLD + li]);
            const T *p = Uin + o;
#pragma unroll
            for (int v = 0; v < NV; v++)
                dst[v] = p[v * P3];
        };
        auto splane = [&](int k) { return su + ((k + 2) & 1) * SUB; };
        auto rplane = [&](int k) { return sring + ((k + 2) & 1) * (NV * NRING); };

        // LF: planes -2 and -1 in LDS before the march (plane -2: the
        // interior columns only, read as the z neighbour of plane -1), the
        // ring of plane 0 in its buffer, outer cells of plane 0 and ring
        // cells of plane 1 in flight.  WENO: plane -2's interior columns in
        // LDS, the ring of plane -1 in its buffer, outer cells of plane -1 and
        // ring cells of plane 0 in flight
        T u0[NV], up[NV], upp[NV], xc[NV];
        {
            T um[NV];
            load(um, -2);
            T *s = splane(-2);
#pragma unroll
            for (int v = 0; v < NV; v++)
                s[v * XS3 + q] = um[v];
        }
        load(u0, -1);
        load(up, 0);
        if constexpr (TWOB) {
            T *s = splane(-1);
#pragma unroll
            for (int v = 0; v < NV; v++)
                s[v * XS3 + q] = u0[v];
            if (isld) {
                T r1[NV];
                load_x(r1, -1);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    s[v * XS3 + xq] = r1[v];
                if (isring) {
                    load_x(r1, 0);
                    T *rb = rplane(0);
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        rb[v * NRING + ri] = r1[v];
                }
            }
            if (isout)
                load_x(xc, 0);
            else if (isring)
                load_x(xc, 1);
            __syncthreads();
        } else {
            if (isout) {
                load_x(xc, -1);
            } else if (isring) {
                T r1[NV];
                load_x(r1, -1);
                T *rb = rplane(-1);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    rb[v * NRING + ri] = r1[v];
                load_x(xc, 0);
            }
        }
        // carried to the next plane: Wc = u - (in-plane flux differences)
        // + dt (sources + in-plane resistive terms), the flux of the face
        // k-1/2, the left state of the face k+1/2, eta J of two planes
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

        // slopes (limiter1) of the cell at in-plane position c of plane k,
        // with its z neighbours um / up
        auto slopes = [&](const T *sc, int c, const T uc[NV], const T um_[NV], const T up_[NV],
                          T (&dl)[3][NV]) {
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const T *row = sc + v * XS3;
                dl[0][v] = limiter<LIM>(uc[v] - row[c - 1], row[c + 1] - uc[v]);
                dl[1][v] = limiter<LIM>(uc[v] - row[c - SY], row[c + SY] - uc[v]);
                dl[2][v] = limiter<LIM>(uc[v] - um_[v], up_[v] - uc[v]);
            }
        };
        // half-step predictor u~ = u - dt/(2dx) sum_d [f(u + D/2) - f(u - D/2)],
        // evaluated optimistically; if any of its face states has rho <= 0
        // or p <= 0 the slopes fall back to zero and u~ = u
        auto predict = [&](const T uc[NV], T (&dl)[3][NV], T (&ut)[NV]) {
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
                    s1[v] = uc[v] + T(0.5) * dl[d][v];
                prim_of(ph, s1, w);
                ok = ok && admissible_w(s1, w);
                flux_w<d>(s1, w, ch2, f1);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    s1[v] = uc[v] - T(0.5) * dl[d][v];
                prim_of(ph, s1, w);
                ok = ok && admissible_w(s1, w);
                flux_w<d>(s1, w, ch2, f2);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    acc[v] += hdt[d] * (f1[v] - f2[v]);
            };
            pred(std::integral_constant<int, 0>{});
            pred(std::integral_constant<int, 1>{});
            pred(std::integral_constant<int, 2>{});
            if (!ok) {
#pragma unroll
                for (int d = 0; d < 3; d++)
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        dl[d][v] = T(0);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    acc[v] = T(0);
                atomicAdd(&a.cnt[0], 1ull);
            }
#pragma unroll
            for (int v = 0; v < NV; v++)
                ut[v] = uc[v] - acc[v];
        };
        // eta J and eta (J x B) of the cell at c from central differences
        auto curl = [&](const T *sc, int c, const T uc[NV], const T um_[NV], const T up_[NV],
                        T (&e)[5], T &qz) {
            const T *bx = sc + BX * XS3, *by = sc + BY * XS3, *bz = sc + BZ * XS3;
            const T dyBz = (bz[c + SY] - bz[c - SY]) * i2d[1];
            const T dzBy = (up_[BY] - um_[BY]) * i2d[2];
            const T dzBx = (up_[BX] - um_[BX]) * i2d[2];
            const T dxBz = (bz[c + 1] - bz[c - 1]) * i2d[0];
            const T dxBy = (by[c + 1] - by[c - 1]) * i2d[0];
            const T dyBx = (bx[c + SY] - bx[c - SY]) * i2d[1];
            const T jx = dyBz - dzBy, jy = dzBx - dxBz, jz = dxBy - dyBx;
            e[0] = eta * jx;
            e[1] = eta * jy;
            e[2] = eta * jz;
            e[3] = eta * (jz * uc[BY] - jy * uc[BZ]);
            e[4] = eta * (jx * uc[BZ] - jz * uc[BX]);
            qz = eta * (jy * uc[BX] - jx * uc[BY]);
        };

        for (int k = -1; k <= NB; ++k) {
            const bool kI = k >= 0 && k < NB;
            T *const sc = splane(k);
            T *const sm = splane(k - 1);
            if constexpr (TWOB) {
                // plane k is in LDS (published before the previous plane's
                // last barrier); prefetch the interior columns of plane k+2
                if (k + 2 <= NB + 1)
                    load(upp, k + 2);
            } else {
                // ---- (A) publish plane k; prefetch plane k+2 (interior,
                //      ring) and k+1 (outer cells)
#pragma unroll
                for (int v = 0; v < NV; v++)
                    sc[v * XS3 + q] = u0[v];
                if (isout) {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        sc[v * XS3 + xq] = xc[v];
                    if (k + 1 <= NB + 1)
                        load_x(xc, k + 1);
                } else if (isring) {
                    const T *rk = rplane(k);
                    T *rn = rplane(k + 1);
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        sc[v * XS3 + xq] = rk[v * NRING + ri];
                        rn[v * NRING + ri] = xc[v];
                    }
                    if (k + 2 <= NB + 1)
                        load_x(xc, k + 2);
                }
                if (k + 2 <= NB + 1)
                    load(upp, k + 2);
                __syncthreads();
            }

            // ---- ring pass: the one face state of each ring cell the
            //      interior reads, and its eta J
            // LF: the wave that runs this plane's ring pass has the most work
            // before the barrier (B); it issues ahead of the other workgroup's
            // wave on its SIMD until then (from the previous plane's barrier
            // (D) on)
            const bool ringw = RING1 && kI && wv == (k & 3);
            if (ringw)
                __builtin_amdgcn_s_setprio(2);
            if (kI && (RING1 ? wv == (k & 3) : isring)) {
                T ur[NV], urm[NV], urp[NV];
                const T *rn = rplane(k + 1);
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    ur[v] = sc[v * XS3 + xqr];
                    urm[v] = sm[v * XS3 + xqr];
                    urp[v] = rn[v * NRING + rir];
                }
                // left state of the face -1/2 (ring at -1) or right state of
                // the face NB-1/2 (ring at NB); a state with rho <= 0 or
                // p <= 0 is replaced by the cell's u~ (LF) or u (WENO)
                T S[NV], ut[NV];
                Prim<T> ws;
                if constexpr (SCH == SCH_LF) {
                    T dl[3][NV];
                    slopes(sc, xqr, ur, urm, urp, dl);
                    predict(ur, dl, ut);
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        const T dv = rdr == 0 ? dl[0][v] : dl[1][v];
                        S[v] = rlr ? ut[v] + T(0.5) * dv : ut[v] - T(0.5) * dv;
                    }
                } else {
                    const int st = rdr == 0 ? 1 : SY;
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        const T *row = sc + v * XS3;
                        T L, R;
                        weno_pair(row[xqr - st], ur[v], row[xqr + st], L, R);
                        S[v] = rlr ? L : R;
                        ut[v] = ur[v];
                    }
                }
                prim_of(ph, S, ws);
                if (!admissible_w(S, ws)) {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        S[v] = ut[v];
                    prim_of(ph, S, ws);
                    atomicAdd(&a.cnt[1], 1ull);
                }
#pragma unroll
                for (int v = 0; v < NV; v++)
                    srf[(rdr * NV + v) * XS3 + xqr] = S[v];
                spr[rdr * XS3 + xqr] = ws.p;
                if constexpr (RESIST) {
                    T e[5], qz;
                    curl(sc, xqr, ur, urm, urp, e, qz);
#pragma unroll
                    for (int i = 0; i < 5; i++)
                        sj[i * XS3 + xqr] = e[i];
                }
            }

            // ---- interior pass: slopes, predictor, face states in the three
            //      dimensions, EGLM sources, eta J
            T Lin[2][NV], pLin[2], Lm[NV], Rm[NV], fmc[NV];
            T pLm = T(1), pRm = T(1);
            T src[4] = {T(0), T(0), T(0), T(0)};
            T jc[3] = {T(0), T(0), T(0)};
            {
                T dl[3][NV], ut[NV];
                // (u0 is this column's cell of plane k; um is read back from LDS)
                T um[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    um[v] = sm[v * XS3 + q];
                if constexpr (SCH == SCH_LF) {
                    slopes(sc, q, u0, um, up, dl);
                    predict(u0, dl, ut);
                } else {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        ut[v] = u0[v];  // the fall-back state of WENO faces
                }
                const int qc[3] = {qx, qy, k};
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    T L[NV], R[NV];
                    Prim<T> wl, wr;
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        if constexpr (SCH == SCH_LF) {
                            L[v] = ut[v] + T(0.5) * dl[d][v];
                            R[v] = ut[v] - T(0.5) * dl[d][v];
                        } else {
                            const T *row = sc + v * XS3;
                            const T m = d == 0 ? row[q - 1] : (d == 1 ? row[q - SY] : um[v]);
                            const T p = d == 0 ? row[q + 1] : (d == 1 ? row[q + SY] : up[v]);
                            weno_pair(m, u0[v], p, L[v], R[v]);
                        }
                    }
                    prim_of(ph, L, wl);
                    prim_of(ph, R, wr);
                    // count a replaced state once, for faces of interior cells
                    bool others = true;
#pragma unroll
                    for (int e = 0; e < 3; e++)
                        if (e != d)
                            others = others && qc[e] >= 0 && qc[e] < NB;
                    if (!admissible_w(L, wl)) {
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            L[v] = ut[v];
                        prim_of(ph, L, wl);
                        if (others && qc[d] < NB)
                            atomicAdd(&a.cnt[1], 1ull);
                    }
                    if (!admissible_w(R, wr)) {
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            R[v] = ut[v];
                        prim_of(ph, R, wr);
                        if (others && qc[d] >= 0)
                            atomicAdd(&a.cnt[1], 1ull);
                    }
                    if (d < 2) {
#pragma unroll
                        for (int v = 0; v < NV; v++) {
                            srf[(d * NV + v) * XS3 + q] = R[v];
                            Lin[d < 2 ? d : 0][v] = L[v];
                        }
                        spr[d * XS3 + q] = wr.p;
                        pLin[d < 2 ? d : 0] = wl.p;
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
                // the flux of the face k-1/2 from registers only: formed here,
                // before the barriers, so that its states die early
                if (k >= 0)
                    face_flux<RS, 2>(Lm_prev, pLm_prev, Rm, pRm, gam, ph.gm1, ch, ch2, fmc);
                // EGLM sources from central differences of u^n
                if (a.eglm && kI) {
                    const T *bx = sc + BX * XS3, *by = sc + BY * XS3, *ps = sc + PSI * XS3;
                    T divb = (bx[q + 1] - bx[q - 1]) * i2d[0];
                    T bgp = u0[BX] * ((ps[q + 1] - ps[q - 1]) * i2d[0]);
                    divb += (by[q + SY] - by[q - SY]) * i2d[1];
                    bgp += u0[BY] * ((ps[q + SY] - ps[q - SY]) * i2d[1]);
                    divb += (up[BZ] - um[BZ]) * i2d[2];
                    bgp += u0[BZ] * ((up[PSI] - um[PSI]) * i2d[2]);
                    src[0] = divb * u0[BX];
                    src[1] = divb * u0[BY];
                    src[2] = divb * u0[BZ];
                    src[3] = bgp;
                }
                if constexpr (RESIST) {
                    T e[5], qz;
                    curl(sc, q, u0, um, up, e, qz);
#pragma unroll
                    for (int i = 0; i < 5; i++)
                        sj[i * XS3 + q] = e[i];
                    jc[0] = e[0];
                    jc[1] = e[1];
                    jc[2] = qz;
                }
            }
            if (ringw)
                __builtin_amdgcn_s_setprio(0);
            __syncthreads();  // (B) face states, their pressures and eta J published

            // ---- LF: publish plane k+1 into the slot of plane k-1, whose
            //      last readers (ring and interior passes) are behind (B);
            //      the barrier (D) below orders it before plane k+1's
            //      passes.  Prefetch the outer cells of plane k+2 and the
            //      ring cells of plane k+3.
            if (TWOB && k + 1 <= NB) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    sm[v * XS3 + q] = up[v];
                if (isout) {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        sm[v * XS3 + xq] = xc[v];
                    if (k + 2 <= NB + 1)
                        load_x(xc, k + 2);
                } else if (isring) {
                    const T *r1 = rplane(k + 1);
                    T *r2 = rplane(k + 2);
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        sm[v * XS3 + xq] = r1[v * NRING + ri];
                        r2[v * NRING + ri] = xc[v];
                    }
                    if (k + 3 <= NB + 1)
                        load_x(xc, k + 3);
                }
            }

            // WENO stage 2: u of the cell finalised in this iteration,
            // requested before the flux phase so that it lands during it
            T ubase[SCH == SCH_WENO2 ? NV : 1];
            if constexpr (SCH == SCH_WENO2) {
                if (k >= 1) {
                    const T *b = (const T *)a.Ubase + (size_t)slot * NV * P3 + (k - 1 + NG) * XS3 + q;
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        ubase[v] = b[v * P3];
                }
            }

            // ---- fluxes: in-plane faces x+1/2, y+1/2 of the interior cells and
            //      the faces -1/2 (ring waves of the -1 sides).  The flux of a
            //      face replaces the right state it was formed from, in the
            //      slot of the cell on the face's right: that slot has one
            //      reader, the lane that forms the flux, so no barrier is
            //      needed between the reads of the states and the writes of
            //      the fluxes
            T fin[2][NV];
            T rin[4] = {T(0), T(0), T(0), T(0)};
            if (kI) {
                T R[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    R[v] = srf[(0 * NV + v) * XS3 + q + 1];
                face_flux<RS, 0>(Lin[0], pLin[0], R, spr[q + 1], gam, ph.gm1, ch, ch2, fin[0]);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    srf[(0 * NV + v) * XS3 + q + 1] = fin[0][v];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    R[v] = srf[(1 * NV + v) * XS3 + q + SY];
                face_flux<RS, 1>(Lin[1], pLin[1], R, spr[XS3 + q + SY], gam, ph.gm1, ch, ch2, fin[1]);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    srf[(1 * NV + v) * XS3 + q + SY] = fin[1][v];
            }
            if (kI && isring && rlo) {
                // the ring cell's own state is the left one, the first
                // interior cell's the right one
                const int qn = xq + (rdim == 0 ? 1 : SY);
                T L[NV], R[NV], f[NV];
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    L[v] = srf[(rdim * NV + v) * XS3 + xq];
                    R[v] = srf[(rdim * NV + v) * XS3 + qn];
                }
                const T pl = spr[rdim * XS3 + xq], pr = spr[rdim * XS3 + qn];
                if (rdim == 0)
                    face_flux<RS, 0>(L, pl, R, pr, gam, ph.gm1, ch, ch2, f);
                else
                    face_flux<RS, 1>(L, pl, R, pr, gam, ph.gm1, ch, ch2, f);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    srf[(rdim * NV + v) * XS3 + qn] = f[v];
                const int fb = a.fbidx[(size_t)slot * 6 + 2 * rdim];
                if (fb >= 0) {
                    const int tt = (rdim == 0 ? ey : ex) + NB * k;
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        put_flux(((size_t)fb * NV + v) * FC + tt, f[v]);
                }
            }
            if constexpr (RESIST) {
                if (kI) {
                    const T *J0 = sj, *J1 = sj + XS3, *J2 = sj + 2 * XS3, *Q0 = sj + 3 * XS3,
                            *Q1 = sj + 4 * XS3;
                    rin[0] = -((J2[q + SY] - J2[q - SY]) * i2d[1]);
                    rin[1] = (J2[q + 1] - J2[q - 1]) * i2d[0];
                    rin[2] = (J0[q + SY] - J0[q - SY]) * i2d[1] - (J1[q + 1] - J1[q - 1]) * i2d[0];
                    rin[3] = (Q0[q + 1] - Q0[q - 1]) * i2d[0] + (Q1[q + SY] - Q1[q - SY]) * i2d[1];
                }
            }
            const bool dom = k >= 0;
            if (kI) {
                // fluxes of block faces shared with another level (reflux):
                // the faces NB-1/2 here, the faces -1/2 in the ring pass
#pragma unroll
                for (int d = 0; d < 2; d++) {
                    const int qd = d == 0 ? qx : qy;
                    if (qd != NB - 1)
                        continue;
                    const int fb = a.fbidx[(size_t)slot * 6 + 2 * d + 1];
                    if (fb < 0)
                        continue;
                    const int tt = (d == 0 ? qy : qx) + NB * k;
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        put_flux(((size_t)fb * NV + v) * FC + tt, fin[d][v]);
                }
            }
            if (dom && (k == 0 || k == NB)) {
                const int fb = a.fbidx[(size_t)slot * 6 + 4 + (k == NB ? 1 : 0)];
                if (fb >= 0) {
                    const int tt = qx + NB * qy;
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        put_flux(((size_t)fb * NV + v) * FC + tt, fmc[v]);
                }
            }
            __syncthreads();  // (D) in-plane face fluxes published
            // LF: the wave that runs the next plane's ring pass takes its
            // raised priority from here, through this plane's finalisation
            if (RING1 && k + 1 < NB && wv == ((k + 1) & 3))
                __builtin_amdgcn_s_setprio(2);

            // ---- finalise plane k-1 with the face k-1/2: z flux difference,
            //      z resistive terms, the Runge-Kutta average (WENO stage 2),
            //      psi damping (MHD-5 integrated exactly, once per step)
            if (dom && k >= 1) {
                T o[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    o[v] = Wc[v] - dtdx[2] * (fmc[v] - fm_prev[v]);
                if constexpr (RESIST) {
                    o[BX] = o[BX] + dt * ((jc[1] - jm2[1]) * i2d[2]);
                    o[BY] = o[BY] - dt * ((jc[0] - jm2[0]) * i2d[2]);
                    o[EN] = o[EN] + dt * ((jc[2] - jm2[2]) * i2d[2]);
                }
                if constexpr (SCH == SCH_WENO2) {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        o[v] = T(0.5) * (ubase[v] + o[v]);
                }
                if constexpr (SCH != SCH_WENO1)
                    o[PSI] = o[PSI] * damp;
#pragma unroll
                for (int v = 0; v < NV; v++)
                    ob[v * P3 + (k - 1 + NG) * XS3 + q] = o[v];
            }
            // ---- start plane k: in-plane flux differences, EGLM sources and
            //      in-plane resistive terms
            if (kI) {
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    T acc = dtdx[0] * (fin[0][v] - srf[(0 * NV + v) * XS3 + q]);
                    acc += dtdx[1] * (fin[1][v] - srf[(1 * NV + v) * XS3 + q]);
                    Wc[v] = sc[v * XS3 + q] - acc;
                }
                if (a.eglm) {
                    Wc[MX] = Wc[MX] - dt * src[0];
                    Wc[MY] = Wc[MY] - dt * src[1];
                    Wc[MZ] = Wc[MZ] - dt * src[2];
                    Wc[EN] = Wc[EN] - dt * src[3];
                }
                if constexpr (RESIST) {
                    Wc[BX] = Wc[BX] + dt * rin[0];
                    Wc[BY] = Wc[BY] + dt * rin[1];
                    Wc[BZ] = Wc[BZ] + dt * rin[2];
                    Wc[EN] = Wc[EN] + dt * rin[3];
                }
            }
            // ---- shift the march-axis registers
#pragma unroll
            for (int v = 0; v < NV; v++) {
                fm_prev[v] = dom ? fmc[v] : T(0);
                Lm_prev[v] = Lm[v];
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

// FP32: compiled for two workgroups per CU (shape 0) or one (shape 1, twice
// the registers); FP64 (148 KB of LDS) for one
template <typename T, bool MIXED, bool RESIST, int SCH, int LIM, int RS>
static hipError_t launch3(const StepArgs &a, int grid, hipStream_t s)
{
    const int g = grid > 0 ? (grid < a.nitems ? grid : a.nitems) : a.nitems;
    if constexpr (sizeof(T) == 4) {
        if (a.shape == 1)
            hipLaunchKernelGGL((k_step3<T, MIXED, RESIST, SCH, LIM, RS, 1>), dim3(g), dim3(NT3), 0,
                               s, a);
        else
            hipLaunchKernelGGL((k_step3<T, MIXED, RESIST, SCH, LIM, RS, 2>), dim3(g), dim3(NT3), 0,
                               s, a);
    } else {
        hipLaunchKernelGGL((k_step3<T, MIXED, RESIST, SCH, LIM, RS, 1>), dim3(g), dim3(NT3), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace mapk
