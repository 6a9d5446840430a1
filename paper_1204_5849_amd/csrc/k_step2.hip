// k_step2.hip -- the block update of 2-D leaf blocks: the TVD-LF step
// (paper Sec. 3.2) or one stage of WENO with TVD Runge-Kutta 2 (Sec. 3.3),
// both directions together (Sec. 3.7), with the EGLM source terms (Sec. 2),
// uniform resistivity (Sec. 3.5) and exact psi damping (the 3-D kernel is in
// k_step3.hpp).
//
// Layout and schedule (gfx950): a workgroup holds BPW blocks, 18 columns
// each (x = -1 .. 16: the interior and the cell on each side whose face
// states feed the block's x faces): 14 blocks in 256 threads, or 7 in 128
// (the launch autotuner picks one).  Threads march along y, one
// row per iteration:
//   * y neighbours (slopes, the half-step flux, the face between rows,
//     source and resistive differences) stay in the thread's registers;
//   * x neighbours are exchanged through LDS one row at a time (state, right
//     face states, face fluxes, eta J); the outer cells x = -2 and x = 17
//     are only loaded, by the first threads, one row ahead.  LF takes two
//     barriers per row, face states published and face fluxes published,
//     and writes the state of row k+1 between the two into the slot of row
//     k-1; the WENO stages publish row k behind a third barrier;
//   * ghost cells are read where the ghost descriptors point (Sec. 4.3): a
//     same-level neighbour's interior in U_in, with periodic wrap or outflow
//     clamping, or the block's own prolongated ghost region, so no copy pass
//     fills same-level ghosts before the update and U_out must not alias
//     U_in;
//   * each face flux is evaluated once; the next row is prefetched from HBM
//     while the current one is processed;
//   * WENO stages take three-cell WENO face states (no predictor); stage 1
//     stores u1 without damping, stage 2 stores (u + u1 + dt L(u1)) / 2, u
//     read from U_base at the cell itself, damps psi, and averages the reflux
//     face fluxes of both stages.
// A persistent grid strides over the leaf list.
#include <type_traits>

#include "cfl.hpp"
#include "kernels.hpp"
#include "physics.hpp"
#include "step_common.hpp"
#include "sched.hpp"
#include "tile.hpp"

namespace mapk {

namespace {
constexpr int XS2 = PD;            // row stride
constexpr int P2 = PD * PD;        // padded tile cells
constexpr int NCOL2 = NB + 2;      // computing columns per block
// the two workgroup shapes: blocks per workgroup and threads
constexpr int nt_of(int bpw) { return bpw == 14 ? 256 : 128; }
// FP32: compiled asking for three waves per SIMD (three 4-wave or six 2-wave
// workgroups per CU); the 14-block shape then takes 168 registers (38
// spilled), the 7-block one keeps two waves per SIMD with a schedule that
// measured 4 % faster on the KH ensemble.  FP64: no hint.
template <typename T>
constexpr int occ_hint(int bpw) { return sizeof(T) == 4 ? (bpw == 14 ? 3 : 6) : 1; }
}  // namespace

template <typename T, bool MIXED, bool RESIST, int SCH, int LIM, int RS, int BPW>
__global__ void __launch_bounds__(nt_of(BPW), occ_hint<T>(BPW)) k_step2(StepArgs a)
{
    constexpr int XS = XS2, P = P2, FC = NB;
    constexpr int NT2 = nt_of(BPW);
    constexpr int NXT2 = 2 * BPW;  // load-only cells (x = -2, x = 17) per row
    static_assert(BPW * NCOL2 <= NT2, "one thread per column");
    constexpr int SUB = BPW * NV * XS;
    // LF: two barriers per row, the next row published between them; WENO
    // stages: a third barrier after publishing row k at the top of its
    // iteration (as in the 3-D kernel)
    constexpr bool TWOB = SCH == SCH_LF;
    __shared__ T su[2 * SUB];             // state of rows k and k-1 (by parity)
    __shared__ T srf[BPW * NV * XS];      // right face states, then fluxes
    __shared__ T spr[BPW * XS];           // pressures of those face states
    __shared__ T sj[RESIST ? BPW * 5 * XS : 1];
    // per thread: where its column (and its load-only cell) reads the row
    // regions -2, -1, the interior (row 0; row k adds k XS), NB, NB+1, as
    // element offsets from Uin (the loads stay in the global address space)
    __shared__ size_t gcol[5 * NT2];
    __shared__ size_t gxc[5 * NXT2];
    // LF with cfl_on: the next cycle's CFL maximum of each block, as the bits
    // of a non-negative double (they order like the values)
    __shared__ unsigned long long scfl[SCH == SCH_LF ? BPW : 1];

    // ---- this thread's column and its extra (load-only) cell
    const int t = threadIdx.x;
    int lb = t / NCOL2;
    const bool lane = lb < BPW;
    int qx = t - lb * NCOL2 - 1;
    if (!lane) {
        lb = 0;
        qx = 0;
    }
    const int q = qx + NG;
    int xq = -1, xlb = 0, ex = 0;
    if (t < NXT2) {
        xlb = t >> 1;
        xq = (t & 1) ? PD - 1 : 0;
        ex = xq - NG;
    }
    const bool inI = lane && qx >= 0 && qx < NB;

    Phys<T, MIXED> ph;
    ph.gamma = (T)a.gamma;
    ph.gm1 = (T)(a.gamma - 1.0);
    ph.gm1d = a.gamma - 1.0;
    const T gam = (T)a.gamma;
    const T *Uin = (const T *)a.Uin;
    T *Uout = (T *)a.Uout;
    T *fbuf = (T *)a.fbuf;
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
        const int li = item * BPW + lb;
        const bool has = lane && li < a.nleaves;
        const int slot = has ? a.leaves[li] : 0;
        const int lix = item * BPW + xlb;
        const bool xhas = xq >= 0 && lix < a.nleaves;
        const int xslot = xhas ? a.leaves[lix] : 0;
        const BlockRec br = a.blk[slot];
        const map_dt rec = a.dt[br.sim];
        const double *dxp = a.lvl_dx + ((size_t)br.sim * (MAXL + 1) + br.level) * 3;
        T dtdx[2], hdt[2], i2d[2];
#pragma unroll
        for (int d = 0; d < 2; d++) {
            double r = rec.dt / dxp[d];
            dtdx[d] = (T)r;
            hdt[d] = (T)(0.5 * r);
            i2d[d] = (T)(0.5 / dxp[d]);
        }
        const T dt = (T)rec.dt, ch = (T)rec.ch, ch2 = (T)(rec.ch * rec.ch), damp = (T)rec.damp;
        const T eta = (T)a.eta;
        T *ob = Uout + (size_t)slot * NV * P;
        // LF with cfl_on: this block's leaf index when the update forms its
        // next CFL maximum (the values below are final for this cycle), -1
        // otherwise; the running maximum and the counts of the cells the
        // CFL pass would count
        const int cfl_l = SCH == SCH_LF && a.cfl_on && has ? a.cfl_leaf[slot] : -1;
        double cfl_m = 0.0;
        unsigned cfl_bad = 0, cfl_nonfin = 0;
        if constexpr (SCH == SCH_LF) {
            if (a.cfl_on && t < BPW)
                scfl[t] = 0ull;
        }

        auto set_src = [&](size_t *tab, int ts, int sl, int cx) {
            const int yr[5] = {-2, -1, 0, NB, NB + 1};
#pragma unroll
            for (int r = 0; r < 5; r++)
                tab[r * ts] = cell_src<2>(a.desc, sl, cx, yr[r], 0);
        };
        // k is the same for the whole workgroup: the region choice is uniform
        auto src_of = [&](const size_t *tab, int ts, int k) -> const T * {
            if (k < 0)
                return Uin + tab[(k + 2) * ts];
            if (k < NB)
                return Uin + tab[2 * ts] + k * XS;
            return Uin + tab[(k - NB + 3) * ts];
        };
        if (has)
            set_src(gcol + t, NT2, slot, qx);
        if (xhas)
            set_src(gxc + t, NXT2, xslot, ex);

        auto load = [&](T(&dst)[NV], int k) {
            if (has) {
                const T *p = src_of(gcol + t, NT2, k);
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
                const T *p = src_of(gxc + t, NXT2, k);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    dst[v] = p[v * P];
            }
        };

        T u0[NV], up[NV], upp[NV], xc[NV];
        {
            // row -2 of the own column: read back as the k-1 row at k = -1
            T um[NV];
            load(um, -2);
            if (lane) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    su[(lb * NV + v) * XS + q] = um[v];
            }
        }
        load(u0, -1);
        load(up, 0);
        load_x(xc, -1);
        if constexpr (TWOB) {
            // LF: row -1 in LDS before the march, the load-only cell of row 0
            // in flight
            T *const s = su + SUB;  // row -1
            if (lane) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    s[(lb * NV + v) * XS + q] = u0[v];
            }
            if (xhas) {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    s[(xlb * NV + v) * XS + xq] = xc[v];
            }
            load_x(xc, 0);
            __syncthreads();
        }
        // carried to the next row: Wc = u - (x flux difference) + dt (sources
        // + x resistive terms), the flux of the face k-1/2 (the y difference
        // is taken as a difference, so a uniform state stays exactly
        // uniform), the left state of the face k+1/2, eta J of two rows
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
            T *const sc = su + ((k + 2) & 1) * SUB;  // row k
            T *const sm = su + ((k + 1) & 1) * SUB;  // row k-1
            auto um = [&](int v) { return sm[(lb * NV + v) * XS + q]; };
            // WENO stage 2: u of the cell finalised in this iteration
            T ubase[SCH == SCH_WENO2 ? NV : 1];
            if constexpr (TWOB) {
                // row k is in LDS (published before the previous row's last
                // barrier); prefetch the own column's row k+2
                if (k + 2 <= NB + 1)
                    load(upp, k + 2);
            } else {
                // ---- (A) publish row k (own column and the load-only cell)
                if (lane) {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        sc[(lb * NV + v) * XS + q] = u0[v];
                }
                if (xhas) {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        sc[(xlb * NV + v) * XS + xq] = xc[v];
                }
                if (k + 2 <= NB + 1)
                    load(upp, k + 2);
                if (k + 1 <= NB + 1)
                    load_x(xc, k + 1);
                if constexpr (SCH == SCH_WENO2) {
                    if (inI && k >= 1 && has) {
                        const T *b = (const T *)a.Ubase + (size_t)slot * NV * P + (k - 1 + NG) * XS + q;
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            ubase[v] = b[v * P];
                    }
                }
                __syncthreads();
            }

            T Lin[NV], pLin = T(1), Lm[NV], Rm[NV], fmc[NV];
            T pLm = T(1), pRm = T(1);
            T src[4] = {T(0), T(0), T(0), T(0)};
            T jc[3] = {T(0), T(0), T(0)};
            // rows -1 and NB only feed the faces between rows: interior columns
            const bool work = lane && (kI || inI);
            if (work) {
                // slopes from the old-time differences (limiter1)
                T dl[2][NV];
                T ut[NV];
                if constexpr (SCH == SCH_LF) {
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        const T *row = sc + (lb * NV + v) * XS;
                        dl[0][v] = limiter<LIM>(u0[v] - row[q - 1], row[q + 1] - u0[v]);
                        dl[1][v] = limiter<LIM>(u0[v] - um(v), up[v] - u0[v]);
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
                    if (!ok) {
#pragma unroll
                        for (int d = 0; d < 2; d++)
#pragma unroll
                            for (int v = 0; v < NV; v++)
                                dl[d][v] = T(0);
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            acc[v] = T(0);
                        if (has)
                            atomicAdd(&a.cnt[0], 1ull);
                    }
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        ut[v] = u0[v] - acc[v];
                } else {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        ut[v] = u0[v];  // the fall-back state of WENO faces
                }
                // face states with the old-time slopes (limiter2) or WENO; a
                // state with rho <= 0 or p <= 0 is replaced by the cell's u~
                // (LF) or u (WENO)
                const int qc[2] = {qx, k};
#pragma unroll
                for (int d = 0; d < 2; d++) {
                    T L[NV], R[NV];
                    Prim<T> wl, wr;
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        if constexpr (SCH == SCH_LF) {
                            L[v] = ut[v] + T(0.5) * dl[d][v];
                            R[v] = ut[v] - T(0.5) * dl[d][v];
                        } else {
                            const T *row = sc + (lb * NV + v) * XS;
                            weno_pair(d == 0 ? row[q - 1] : um(v), u0[v], d == 0 ? row[q + 1] : up[v],
                                      L[v], R[v]);
                        }
                    }
                    prim_of(ph, L, wl);
                    prim_of(ph, R, wr);
                    // count a replaced state once, for faces of interior cells
                    const bool others = qc[1 - d] >= 0 && qc[1 - d] < NB;
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
                    if (d == 0) {
#pragma unroll
                        for (int v = 0; v < NV; v++) {
                            srf[(lb * NV + v) * XS + q] = R[v];
                            Lin[v] = L[v];
                        }
                        spr[lb * XS + q] = wr.p;
                        pLin = wl.p;
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
                // the flux of the face k-1/2 from registers only, formed
                // before the barriers so that its states die early
                if (inI && k >= 0)
                    face_flux<RS, 1>(Lm_prev, pLm_prev, Rm, pRm, gam, ph.gm1, ch, ch2, fmc);
                // EGLM sources from central differences of u^n
                if (a.eglm && inI && kI) {
                    const T *bx = sc + (lb * NV + BX) * XS;
                    const T *ps = sc + (lb * NV + PSI) * XS;
                    T divb = (bx[q + 1] - bx[q - 1]) * i2d[0];
                    T bgp = u0[BX] * ((ps[q + 1] - ps[q - 1]) * i2d[0]);
                    divb += (up[BY] - um(BY)) * i2d[1];
                    bgp += u0[BY] * ((up[PSI] - um(PSI)) * i2d[1]);
                    src[0] = divb * u0[BX];
                    src[1] = divb * u0[BY];
                    src[2] = divb * u0[BZ];
                    src[3] = bgp;
                }
                // resistivity: eta J and eta (J x B) on this row
                if constexpr (RESIST) {
                    const T *by = sc + (lb * NV + BY) * XS, *bz = sc + (lb * NV + BZ) * XS;
                    const T dyBz = (up[BZ] - um(BZ)) * i2d[1];
                    const T dxBz = (bz[q + 1] - bz[q - 1]) * i2d[0];
                    const T dxBy = (by[q + 1] - by[q - 1]) * i2d[0];
                    const T dyBx = (up[BX] - um(BX)) * i2d[1];
                    const T jx = dyBz, jy = -dxBz, jz = dxBy - dyBx;
                    const T ejx = eta * jx, ejy = eta * jy, ejz = eta * jz;
                    const T qx_ = eta * (jz * u0[BY] - jy * u0[BZ]);
                    const T qy_ = eta * (jx * u0[BZ] - jz * u0[BX]);
                    T *J = sj + lb * 5 * XS;
                    J[0 * XS + q] = ejx;
                    J[1 * XS + q] = ejy;
                    J[2 * XS + q] = ejz;
                    J[3 * XS + q] = qx_;
                    J[4 * XS + q] = qy_;
                    jc[0] = ejx;
                    jc[1] = ejz;
                    jc[2] = qy_;
                }
            }
            __syncthreads();  // (B) right face states, their pressures and eta J published

            // ---- LF: publish row k+1 into the slot of row k-1, whose last
            //      readers are behind (B); the barrier (D) below orders it
            //      before row k+1's pass.  Prefetch the load-only cell of
            //      row k+2.
            if (TWOB && k + 1 <= NB) {
                if (lane) {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        sm[(lb * NV + v) * XS + q] = up[v];
                }
                if (xhas) {
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        sm[(xlb * NV + v) * XS + xq] = xc[v];
                }
                if (k + 2 <= NB + 1)
                    load_x(xc, k + 2);
            }

            // ---- fluxes of the x faces of row k.  The flux of a face replaces
            //      the right state it was formed from, in the slot of the cell
            //      on the face's right: that slot has one reader, the lane that
            //      forms the flux, so no barrier is needed between the reads of
            //      the states and the writes of the fluxes
            T fin[NV];
            T rin[3] = {T(0), T(0), T(0)};
            const bool dof = kI && lane && qx >= -1 && qx < NB;
            if (dof) {
                T R[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    R[v] = srf[(lb * NV + v) * XS + q + 1];
                face_flux<RS, 0>(Lin, pLin, R, spr[lb * XS + q + 1], gam, ph.gm1, ch, ch2, fin);
#pragma unroll
                for (int v = 0; v < NV; v++)
                    srf[(lb * NV + v) * XS + q + 1] = fin[v];
            }
            if constexpr (RESIST) {
                if (inI && kI) {
                    const T *J = sj + lb * 5 * XS;
                    const T *J1 = J + XS, *J2 = J + 2 * XS, *Q0 = J + 3 * XS;
                    rin[0] = (J2[q + 1] - J2[q - 1]) * i2d[0];
                    rin[1] = (J1[q + 1] - J1[q - 1]) * i2d[0];
                    rin[2] = (Q0[q + 1] - Q0[q - 1]) * i2d[0];
                }
            }
            const bool dom = inI && k >= 0;
            // fluxes of block faces shared with another level (reflux)
            if (has) {
                if (dof && (qx == -1 || qx == NB - 1)) {
                    const int fb = a.fbidx[(size_t)slot * 6 + (qx == -1 ? 0 : 1)];
                    if (fb >= 0) {
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            put_flux(((size_t)fb * NV + v) * FC + k, fin[v]);
                    }
                }
                if (dom && (k == 0 || k == NB)) {
                    const int fb = a.fbidx[(size_t)slot * 6 + 2 + (k == NB ? 1 : 0)];
                    if (fb >= 0) {
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            put_flux(((size_t)fb * NV + v) * FC + qx, fmc[v]);
                    }
                }
            }
            __syncthreads();  // (D) x face fluxes published

            // ---- finalise row k-1 with the face k-1/2: y flux difference,
            //      y resistive terms, the Runge-Kutta average (WENO stage 2),
            //      psi damping (MHD-5 integrated exactly, once per step)
            if (dom && k >= 1 && has) {
                T o[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    o[v] = Wc[v] - dtdx[1] * (fmc[v] - fm_prev[v]);
                if constexpr (RESIST) {
                    o[BX] = o[BX] - dt * ((jc[1] - jm2[1]) * i2d[1]);
                    o[BZ] = o[BZ] + dt * ((jc[0] - jm2[0]) * i2d[1]);
                    o[EN] = o[EN] + dt * ((jc[2] - jm2[2]) * i2d[1]);
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
                    ob[v * P + (k - 1 + NG) * XS + q] = o[v];
                if (cfl_l >= 0) {
                    double u[NV];
                    bool fin = true;
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        u[v] = (double)o[v];
                        fin = fin && isfinite(u[v]);
                    }
                    if (!fin) {
                        cfl_nonfin++;
                    } else {
                        double pr;
                        bool b;
                        const double sp = cfl_speed<2>(u, a.gamma, pr, b);
                        if (b)
                            cfl_bad++;
                        cfl_m = sp > cfl_m ? sp : cfl_m;
                    }
                }
            }
            // ---- start row k: x flux difference, EGLM sources and x
            //      resistive terms
            if (inI && kI) {
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const T acc = dtdx[0] * (fin[v] - srf[(lb * NV + v) * XS + q]);
                    Wc[v] = sc[(lb * NV + v) * XS + q] - acc;
                }
                if (a.eglm) {
                    Wc[MX] = Wc[MX] - dt * src[0];
                    Wc[MY] = Wc[MY] - dt * src[1];
                    Wc[MZ] = Wc[MZ] - dt * src[2];
                    Wc[EN] = Wc[EN] - dt * src[3];
                }
                if constexpr (RESIST) {
                    Wc[BY] = Wc[BY] + dt * rin[0];
                    Wc[BZ] = Wc[BZ] - dt * rin[1];
                    Wc[EN] = Wc[EN] + dt * rin[2];
                }
            }
            // ---- shift the march-axis registers
#pragma unroll
            for (int v = 0; v < NV; v++) {
                fm_prev[v] = dom ? fmc[v] : T(0);
                Lm_prev[v] = work ? Lm[v] : T(0);
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
        if constexpr (SCH == SCH_LF) {
            if (a.cfl_on) {
                // the block's maximum over its columns, then one lane per
                // block writes it where the CFL pass would
                if (cfl_l >= 0 && inI) {
                    atomicMax(&scfl[lb], (unsigned long long)__double_as_longlong(cfl_m));
                    if (cfl_bad)
                        atomicAdd(&a.cnt[2], (unsigned long long)cfl_bad);
                    if (cfl_nonfin)
                        atomicAdd(&a.cnt[3], (unsigned long long)cfl_nonfin);
                }
                __syncthreads();
                if (t < BPW) {
                    const int lj = item * BPW + t;
                    if (lj < a.nleaves) {
                        const int cl = a.cfl_leaf[a.leaves[lj]];
                        if (cl >= 0)
                            a.cfl_part[cl] = __longlong_as_double((long long)scfl[t]);
                    }
                }
            }
        }
        __syncthreads();  // LDS reuse by the next work item
    }
}

template <typename T, bool MIXED, bool RESIST, int SCH, int LIM, int RS>
static hipError_t launch2(const StepArgs &a, int grid, hipStream_t s)
{
    const int g = grid > 0 ? (grid < a.nitems ? grid : a.nitems) : a.nitems;
    if (a.shape == 1)
        hipLaunchKernelGGL((k_step2<T, MIXED, RESIST, SCH, LIM, RS, 7>), dim3(g), dim3(nt_of(7)), 0,
                           s, a);
    else
        hipLaunchKernelGGL((k_step2<T, MIXED, RESIST, SCH, LIM, RS, 14>), dim3(g), dim3(nt_of(14)),
                           0, s, a);
    return hipGetLastError();
}

// LF: one instance per limiter; WENO stages use no limiter
template <typename T, bool MIXED, bool RESIST, int RS>
static hipError_t launch2_sch(int sch, const StepArgs &a, int grid, hipStream_t s)
{
    if (sch == SCH_WENO1)
        return launch2<T, MIXED, RESIST, SCH_WENO1, MAP_MINMOD, RS>(a, grid, s);
    if (sch == SCH_WENO2)
        return launch2<T, MIXED, RESIST, SCH_WENO2, MAP_MINMOD, RS>(a, grid, s);
    if (a.limiter == MAP_MINMOD)
        return launch2<T, MIXED, RESIST, SCH_LF, MAP_MINMOD, RS>(a, grid, s);
    if (a.limiter == MAP_VANLEER)
        return launch2<T, MIXED, RESIST, SCH_LF, MAP_VANLEER, RS>(a, grid, s);
    return launch2<T, MIXED, RESIST, SCH_LF, MAP_PAPER_PHI, RS>(a, grid, s);
}

template <typename T, bool MIXED, bool RESIST>
static hipError_t launch2_rs(int sch, const StepArgs &a, int grid, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    if (a.riemann == MAP_HLLC)
        return launch2_sch<T, MIXED, RESIST, MAP_HLLC>(sch, a, grid, s);
    return launch2_sch<T, MIXED, RESIST, MAP_RUSANOV>(sch, a, grid, s);
}

int step_blocks_per_group(int ndim, int scheme, int shape)
{
    if (scheme == MAP_MMC || ndim == 3)
        return 1;
    return shape == 1 ? 7 : 14;
}

hipError_t launch_step2(bool fp64, bool resist, int sch, const StepArgs &a, int grid, hipStream_t s)
{
    if (fp64)
        return resist ? launch2_rs<double, false, true>(sch, a, grid, s)
                      : launch2_rs<double, false, false>(sch, a, grid, s);
    return resist ? launch2_rs<float, true, true>(sch, a, grid, s)
                  : launch2_rs<float, true, false>(sch, a, grid, s);
}

}  // namespace mapk
