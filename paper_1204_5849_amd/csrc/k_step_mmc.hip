// k_step_mmc.hip -- the modified MacCormack block update (paper Sec. 3.1) on
// 2-D blocks: Lax-Friedrichs flux splitting f+- = (f +- alpha u)/2 with the
// global alpha (c_h on the GLM pair), predictor u~ from h = f+_i + f-_{i+1},
// and the flux-limited correction built from g+ and g-, all directions
// together (Sec. 3.7), followed by the same EGLM sources, resistive terms
// and psi damping as the LF update.  (3-D blocks: k_step_mmc3.hip.)
//
// One workgroup per block (256 threads).  The padded tile of u^n is staged
// in LDS first, its ghost cells read where the ghost descriptors point (a
// same-level neighbour's interior in U_in, or the block's own prolongated
// ghosts), so U_out must not alias U_in.  Split fluxes of one dimension are
// staged in LDS at a time; the split fluxes of the last predictor dimension
// are reused by the first corrector dimension.
#include "kernels.hpp"
#include "physics.hpp"
#include "sched.hpp"
#include "tile.hpp"

namespace mapk {

namespace {
constexpr int T2 = PD * PD;     // padded cells (400)
constexpr int E2 = (NB + 2) * (NB + 2);  // E region (324)
constexpr int F2 = (NB + 1) * NB;        // faces of one dimension (272)
constexpr int NT = 256;

__device__ __forceinline__ int pidx(int x, int y) { return (y + NG) * PD + (x + NG); }
}  // namespace

template <typename T, bool MIXED, int LIM>
__global__ void __launch_bounds__(NT) k_step_mmc2(StepArgs a)
{
    __shared__ T sfp[NV * T2], sfm[NV * T2];
    __shared__ T stp[NV * E2], stm[NV * E2];
    __shared__ T sfh[NV * F2];
    __shared__ T su[NV * T2];

    Phys<T, MIXED> ph;
    ph.gamma = (T)a.gamma;
    ph.gm1 = (T)(a.gamma - 1.0);
    ph.gm1d = a.gamma - 1.0;
    const T *Uin = (const T *)a.Uin;
    T *Uout = (T *)a.Uout;
    T *fbuf = (T *)a.fbuf;
    const int t = threadIdx.x;

    // neighbouring blocks on one XCD, so that the ghost cells read from
    // neighbours come from that XCD's L2
    int first, stride, end;
    xcd_range(a.nitems, first, stride, end);
    for (int item = first; item < end; item += stride) {
        if (item >= a.nleaves)
            break;
        const int slot = a.leaves[item];
        const BlockRec br = a.blk[slot];
        const map_dt rec = a.dt[br.sim];
        const double *dxp = a.lvl_dx + ((size_t)br.sim * (MAXL + 1) + br.level) * 3;
        T dtdx[2], i2d[2];
        for (int d = 0; d < 2; d++) {
            dtdx[d] = (T)(rec.dt / dxp[d]);
            i2d[d] = (T)(0.5 / dxp[d]);
        }
        const T dt = (T)rec.dt, ch = (T)rec.ch, ch2 = (T)(rec.ch * rec.ch), damp = (T)rec.damp;
        const T alpha = (T)rec.alpha;
        T *ob = Uout + (size_t)slot * NV * T2;
        for (int c = t; c < T2; c += NT) {
            const T *p = Uin + cell_src<2>(a.desc, slot, c % PD - NG, c / PD - NG, 0);
#pragma unroll
            for (int v = 0; v < NV; v++)
                su[v * T2 + c] = p[v * T2];
        }
        __syncthreads();
        const T *ub = su;

        // split fluxes of u along D on the padded tile -> sfp, sfm
        auto split_u = [&](auto dc) {
            constexpr int D = decltype(dc)::value;
            for (int c = t; c < T2; c += NT) {
                T u[NV], F[NV];
#pragma unroll
                for (int v = 0; v < NV; v++)
                    u[v] = ub[v * T2 + c];
                ph.template flux<D, false>(u, ch2, F);
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    T al = (v == BX + D || v == PSI) ? ch : alpha;
                    sfp[v * T2 + c] = T(0.5) * (F[v] + al * u[v]);
                    sfm[v * T2 + c] = T(0.5) * (F[v] - al * u[v]);
                }
            }
        };

        // ---- predictor on E: u~ = u - sum_d dt/dx_d (h_{i+1/2} - h_{i-1/2})
        T term[2][2][NV];  // [own E cell][dim][var]
        auto pred_dim = [&](auto dc) {
            constexpr int D = decltype(dc)::value;
            const int s = D == 0 ? 1 : PD;
            for (int j = 0; j < 2; j++) {
                int e = t + j * NT;
                if (e >= E2)
                    continue;
                int c = pidx(e % (NB + 2) - 1, e / (NB + 2) - 1);
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    T hp = sfp[v * T2 + c] + sfm[v * T2 + c + s];
                    T hm = sfp[v * T2 + c - s] + sfm[v * T2 + c];
                    term[j][D][v] = dtdx[D] * (hp - hm);
                }
            }
        };
        split_u(std::integral_constant<int, 0>{});
        __syncthreads();
        pred_dim(std::integral_constant<int, 0>{});
        __syncthreads();
        split_u(std::integral_constant<int, 1>{});
        __syncthreads();
        pred_dim(std::integral_constant<int, 1>{});
        T ut[2][NV];
        for (int j = 0; j < 2; j++) {
            int e = t + j * NT;
            if (e >= E2)
                continue;
            int c = pidx(e % (NB + 2) - 1, e / (NB + 2) - 1);
#pragma unroll
            for (int v = 0; v < NV; v++)
                ut[j][v] = ub[v * T2 + c] - (term[j][0][v] + term[j][1][v]);
        }

        // ---- corrector, dimension y first (its split fluxes of u are in LDS)
        T div[2][NV];  // per dimension, for the own interior cell
        const int ix = t % NB, iy = t / NB;
        auto corr_dim = [&](auto dc, bool need_split) {
            constexpr int D = decltype(dc)::value;
            const int s = D == 0 ? 1 : PD;
            if (need_split) {
                __syncthreads();
                split_u(dc);
            }
            for (int j = 0; j < 2; j++) {
                int e = t + j * NT;
                if (e >= E2)
                    continue;
                T F[NV];
                ph.template flux<D, false>(ut[j], ch2, F);
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    T al = (v == BX + D || v == PSI) ? ch : alpha;
                    stp[v * E2 + e] = T(0.5) * (F[v] + al * ut[j][v]);
                    stm[v * E2 + e] = T(0.5) * (F[v] - al * ut[j][v]);
                }
            }
            __syncthreads();
            // faces c+1/2 with c_D in [-1, NB), the other coordinate interior
            for (int j = 0; j < 2; j++) {
                int f = t + j * NT;
                if (f >= F2)
                    continue;
                int x, y;
                if (D == 0) {
                    x = f % (NB + 1) - 1;
                    y = f / (NB + 1);
                } else {
                    x = f % NB;
                    y = f / NB - 1;
                }
                const int c = pidx(x, y);
                const int se = D == 0 ? 1 : NB + 2;
                const int ce = (y + 1) * (NB + 2) + (x + 1);
                T fh[NV];
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const T *FP = sfp + v * T2, *FM = sfm + v * T2;
                    const T *TP = stp + v * E2, *TM = stm + v * E2;
                    T h = FP[c] + FM[c + s];
                    T gp_m = TP[ce] - FP[c - s];
                    T gp_p = TP[ce + se] - FP[c];
                    T gm_p = FM[c + s] - TM[ce];
                    T gm_pp = FM[c + 2 * s] - TM[ce + se];
                    fh[v] = h + T(0.5) * (limiter<LIM>(gp_m, gp_p) - limiter<LIM>(gm_pp, gm_p));
                    sfh[v * F2 + f] = fh[v];
                }
                // block faces shared with another level (reflux)
                const int cd = D == 0 ? x : y;
                const int side = cd == -1 ? 0 : (cd == NB - 1 ? 1 : -1);
                if (side >= 0) {
                    const int fb = a.fbidx[(size_t)slot * 6 + 2 * D + side];
                    if (fb >= 0) {
                        const int tt = D == 0 ? y : x;
#pragma unroll
                        for (int v = 0; v < NV; v++)
                            fbuf[((size_t)fb * NV + v) * NB + tt] = fh[v];
                    }
                }
            }
            __syncthreads();
            {
                // own interior cell (ix, iy): faces c-1/2 and c+1/2
                int fp_, fm_;
                if (D == 0) {
                    fp_ = iy * (NB + 1) + (ix + 1);
                    fm_ = iy * (NB + 1) + ix;
                } else {
                    fp_ = (iy + 1) * NB + ix;
                    fm_ = iy * NB + ix;
                }
#pragma unroll
                for (int v = 0; v < NV; v++)
                    div[D][v] = dtdx[D] * (sfh[v * F2 + fp_] - sfh[v * F2 + fm_]);
            }
        };
        corr_dim(std::integral_constant<int, 1>{}, false);
        corr_dim(std::integral_constant<int, 0>{}, true);

        // ---- update, EGLM sources from u^n, psi damping
        {
            const int c = pidx(ix, iy);
            T o[NV];
#pragma unroll
            for (int v = 0; v < NV; v++)
                o[v] = ub[v * T2 + c] - (div[0][v] + div[1][v]);
            if (a.eglm) {
                const T *bx = ub + BX * T2, *by = ub + BY * T2, *ps = ub + PSI * T2;
                T divb = (bx[c + 1] - bx[c - 1]) * i2d[0];
                divb += (by[c + PD] - by[c - PD]) * i2d[1];
                T bgp = bx[c] * ((ps[c + 1] - ps[c - 1]) * i2d[0]);
                bgp += by[c] * ((ps[c + PD] - ps[c - PD]) * i2d[1]);
                o[MX] = o[MX] - dt * (divb * bx[c]);
                o[MY] = o[MY] - dt * (divb * by[c]);
                o[MZ] = o[MZ] - dt * (divb * ub[BZ * T2 + c]);
                o[EN] = o[EN] - dt * bgp;
            }
            // resistive terms -curl(eta J) and -div((eta J) x B) (Sec. 3.5)
            // from central differences of u^n; in 2-D the z derivatives vanish
            if (a.eta > 0.0) {
                const T eta = (T)a.eta;
                const T *bx = ub + BX * T2, *by = ub + BY * T2, *bz = ub + BZ * T2;
                // eta J and the x, y rows of eta (J x B) at padded index e
                auto ej = [&](int e, T (&r)[5]) {
                    const T jx = (bz[e + PD] - bz[e - PD]) * i2d[1];
                    const T jy = -((bz[e + 1] - bz[e - 1]) * i2d[0]);
                    const T jz = (by[e + 1] - by[e - 1]) * i2d[0] - (bx[e + PD] - bx[e - PD]) * i2d[1];
                    r[0] = eta * jx;
                    r[1] = eta * jy;
                    r[2] = eta * jz;
                    r[3] = eta * (jz * by[e] - jy * bz[e]);
                    r[4] = eta * (jx * bz[e] - jz * bx[e]);
                };
                T xm[5], xp[5], ym[5], yp[5];
                ej(c - 1, xm);
                ej(c + 1, xp);
                ej(c - PD, ym);
                ej(c + PD, yp);
                o[BX] = o[BX] + dt * (-((yp[2] - ym[2]) * i2d[1]));
                o[BY] = o[BY] + dt * ((xp[2] - xm[2]) * i2d[0]);
                o[BZ] = o[BZ] + dt * ((yp[0] - ym[0]) * i2d[1] - (xp[1] - xm[1]) * i2d[0]);
                o[EN] = o[EN] + dt * ((xp[3] - xm[3]) * i2d[0] + (yp[4] - ym[4]) * i2d[1]);
            }
            o[PSI] = o[PSI] * damp;
#pragma unroll
            for (int v = 0; v < NV; v++)
                ob[v * T2 + c] = o[v];
        }
        __syncthreads();
    }
}

template <typename T, bool MIXED, int LIM>
static void launch_mmc(const StepArgs &a, int g, hipStream_t s)
{
    hipLaunchKernelGGL((k_step_mmc2<T, MIXED, LIM>), dim3(g), dim3(NT), 0, s, a);
}

template <typename T, bool MIXED>
static void launch_mmc_lim(const StepArgs &a, int g, hipStream_t s)
{
    if (a.limiter == MAP_MINMOD)
        launch_mmc<T, MIXED, MAP_MINMOD>(a, g, s);
    else if (a.limiter == MAP_VANLEER)
        launch_mmc<T, MIXED, MAP_VANLEER>(a, g, s);
    else
        launch_mmc<T, MIXED, MAP_PAPER_PHI>(a, g, s);
}

hipError_t launch_step_mmc(int ndim, bool fp64, const StepArgs &a, double, int grid, hipStream_t s)
{
    if (ndim == 3)
        return launch_step_mmc3(fp64, a.eta > 0.0, a, grid, s);
    if (a.nitems <= 0)
        return hipSuccess;
    int g = grid > 0 ? (grid < a.nitems ? grid : a.nitems) : a.nitems;
    if (fp64)
        launch_mmc_lim<double, false>(a, g, s);
    else
        launch_mmc_lim<float, true>(a, g, s);
    return hipGetLastError();
}

}  // namespace mapk
