// k_cond.hip -- one sub-step of the thermal-conduction subcycle (paper
// Sec. 3.4): the energy alone advances by the explicit conduction scheme,
// isotropic or along the magnetic field, with the other variables frozen.
//
// Two launches per sub-step, around the energy-only boundary passes:
//   * conduct: one workgroup per leaf marches along z (3-D) with a window of
//     four 18 x 18 planes in LDS (the interior and the first ring of ghost
//     cells, edges and corners included): each plane is gathered where the
//     ghost descriptors point, its T = p / rho, kappa = kappa0 T^n and, along
//     the field, B are formed once per cell, and every interior cell then
//     takes the fluxes through its six faces from LDS.  The new energy goes to
//     the energy plane of a scratch state (the update reads neighbours' old
//     values), the fluxes of faces shared with another level to the reflux
//     buffer;
//   * commit: the new energy of every leaf cell back into U.
// Arithmetic is FP64 for both state precisions and follows the written
// order (no contraction).
#include "kernels.hpp"
#include "physics.hpp"
#include "tile.hpp"

#pragma clang fp contract(off)

namespace mapk {

namespace {
constexpr int NTC = 256;
constexpr int RW = NB + 2;      // ring width: cells -1 .. NB
constexpr int RP = RW * RW;     // cells of one window plane
constexpr int NWIN = 4;         // window planes (z-1, z, z+1 and the one being loaded)
}  // namespace

// one window plane: T, kappa and (along the field) the field of the cells
// (x, y) in [-1, NB]^2 at one z
struct CondPlane {
    double T[RP], K[RP], B[3][RP];
};

template <int NDIM, typename T, int MODE>
__device__ __forceinline__ void cond_gather(const CondArgs &a, const T *U, int slot, int z,
                                            CondPlane &pl, double gm1)
{
    constexpr int P = tile_cells<NDIM>();
    for (int i = threadIdx.x; i < RP; i += NTC) {
        const int x = i % RW - 1, y = i / RW - 1;
        const size_t o = cell_src<NDIM>(a.desc, slot, x, y, z);
        double u[EN + 1];
#pragma unroll
        for (int k = 0; k <= EN; k++)
            u[k] = (double)U[o + (size_t)k * P];
        const double ir = 1.0 / u[RHO];
        const double vx = u[MX] * ir, vy = u[MY] * ir, vz = u[MZ] * ir;
        const double ke = 0.5 * (u[MX] * vx + u[MY] * vy + u[MZ] * vz);
        const double me = 0.5 * (u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ]);
        const double Tt = gm1 * (u[EN] - ke - me) / u[RHO];
        pl.T[i] = Tt;
        pl.K[i] = kappa_of(a.kappa0, a.khalf, Tt);
        if constexpr (MODE == MAP_COND_FIELD) {
            pl.B[0][i] = u[BX];
            pl.B[1][i] = u[BY];
            pl.B[2][i] = u[BZ];
        }
    }
}

// energy flux along +d through the face between cell c (index ic of plane
// pc) and its +d neighbour (index in of plane pn), F = -(kappa grad T)_d:
// the face kappa is the geometric mean of the two cells'; isotropic,
// F = -kappa_f (T_n - T_c)/dx_d; along the field, F = -kappa_f b_d (b . grad T)
// with b from the mean of the two cells' fields and grad T at the face: the
// difference across it along d, and along each other dimension e the mean
// of the two cells' central differences (planes pcm/pcp and pnm/pnp hold
// the z neighbours of c and n; zero where the face field vanishes)
template <int NDIM, int MODE>
__device__ __forceinline__ double face_flux_c(const CondPlane *pc, int ic, const CondPlane *pn,
                                              int in, int d, const CondPlane *pcm,
                                              const CondPlane *pcp, const CondPlane *pnm,
                                              const CondPlane *pnp, const double *dxp)
{
    const double kf = sqrt(pc->K[ic] * pn->K[in]);
    const double gd = (pn->T[in] - pc->T[ic]) / dxp[d];
    if constexpr (MODE == MAP_COND_ISO) {
        return -(kf * gd);
    } else {
        double Bf[3], bb = 0.0;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            Bf[j] = 0.5 * (pc->B[j][ic] + pn->B[j][in]);
            bb += Bf[j] * Bf[j];
        }
        if (!(bb > 0.0))
            return 0.0;
        double bg = 0.0;
#pragma unroll
        for (int e = 0; e < 3; e++) {
            double g;
            if (e == d) {
                g = gd;
            } else if (e == 2 && NDIM == 3) {
                g = ((pcp->T[ic] - pcm->T[ic]) + (pnp->T[in] - pnm->T[in])) / (4.0 * dxp[e]);
            } else if (e < 2) {
                const int s = e == 0 ? 1 : RW;
                g = ((pc->T[ic + s] - pc->T[ic - s]) + (pn->T[in + s] - pn->T[in - s])) /
                    (4.0 * dxp[e]);
            } else {
                g = 0.0;
            }
            bg += Bf[e] * g;
        }
        return -(kf * Bf[d] * bg / bb);
    }
}

template <int NDIM, typename T, int MODE>
__global__ void __launch_bounds__(NTC) k_conduct(CondArgs a)
{
    constexpr int P = tile_cells<NDIM>();
    constexpr int FC = NDIM == 3 ? NB * NB : NB;
    constexpr int NW = NDIM == 3 ? NWIN : 1;
    __shared__ CondPlane win[NW];
    const T *U = (const T *)a.U;
    T *S = (T *)a.S;
    T *fbuf = (T *)a.fbuf;
    const double gm1 = a.gamma - 1.0;
    const int t = threadIdx.x;
    const int qx = t % NB, qy = t / NB;  // this thread's interior column (3-D)
    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const int slot = a.list[item];
        const BlockRec br = a.blk[slot];
        const map_dt rec = a.dt[br.sim];
        if (a.sub >= rec.nsub)
            continue;
        const double *dxp = a.lvl_dx + ((size_t)br.sim * (MAXL + 1) + br.level) * 3;
        const size_t base = (size_t)slot * NV * P;
        // update of one interior cell from the window planes of z-1, z, z+1
        // (in 2-D all three are the one plane)
        auto cell = [&](int x, int y, int z, const CondPlane *pm, const CondPlane *p0,
                        const CondPlane *pp) {
            const int ic = (y + 1) * RW + x + 1;
            const int q[3] = {x, y, z};
            double acc = 0.0;
#pragma unroll
            for (int d = 0; d < NDIM; d++) {
                double fp, fm;
                if (d < 2) {
                    const int s = d == 0 ? 1 : RW;
                    fp = face_flux_c<NDIM, MODE>(p0, ic, p0, ic + s, d, pm, pp, pm, pp, dxp);
                    fm = face_flux_c<NDIM, MODE>(p0, ic - s, p0, ic, d, pm, pp, pm, pp, dxp);
                } else {
                    // z faces: the transverse gradients are in-plane, so the
                    // z-neighbour planes are not read
                    fp = face_flux_c<NDIM, MODE>(p0, ic, pp, ic, d, p0, p0, pp, pp, dxp);
                    fm = face_flux_c<NDIM, MODE>(pm, ic, p0, ic, d, pm, pm, p0, p0, dxp);
                }
                acc += (fp - fm) / dxp[d];
                // faces shared with leaves of another level, for reflux
                const int side = q[d] == 0 ? 0 : (q[d] == NB - 1 ? 1 : -1);
                if (side >= 0) {
                    const int fb = a.fbidx[(size_t)slot * 6 + 2 * d + side];
                    if (fb >= 0) {
                        const int tt = NDIM == 3 ? (d == 0 ? y : x) + NB * (d == 2 ? y : z)
                                                 : (d == 0 ? y : x);
                        fbuf[((size_t)fb * NV + EN) * FC + tt] = (T)(side ? fp : fm);
                    }
                }
            }
            const int c = lin<NDIM>(x, y, z);
            const double e = (double)U[base + (size_t)EN * P + c];
            S[base + (size_t)EN * P + c] = (T)(e - rec.dt_sub * acc);
        };
        if constexpr (NDIM == 2) {
            cond_gather<2, T, MODE>(a, U, slot, 0, win[0], gm1);
            __syncthreads();
            for (int i = t; i < NB * NB; i += NTC)
                cell(i % NB, i / NB, 0, &win[0], &win[0], &win[0]);
            __syncthreads();
        } else {
            // window slot of plane p: (p + 1) mod 4; planes -1 .. NB
            auto W = [&](int p) { return &win[(p + 1) & (NWIN - 1)]; };
            for (int p = -1; p <= 1; p++)
                cond_gather<3, T, MODE>(a, U, slot, p, *W(p), gm1);
            __syncthreads();
            for (int z = 0; z < NB; z++) {
                if (z + 2 <= NB)
                    cond_gather<3, T, MODE>(a, U, slot, z + 2, *W(z + 2), gm1);
                // plane z+2 loads into the slot plane z-2 left while plane z
                // is computed from z-1, z and z+1
                cell(qx, qy, z, W(z - 1), W(z), W(z + 1));
                __syncthreads();
            }
        }
    }
}

template <int NDIM, typename T>
__global__ void __launch_bounds__(NTC) k_cond_commit(CondArgs a)
{
    constexpr int P = tile_cells<NDIM>();
    constexpr int NI = NDIM == 3 ? NB * NB * NB : NB * NB;
    T *U = (T *)a.U;
    const T *S = (const T *)a.S;
    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const int slot = a.list[item];
        if (a.sub >= a.dt[a.blk[slot].sim].nsub)
            continue;
        const size_t e0 = (size_t)slot * NV * P + (size_t)EN * P;
        for (int i = threadIdx.x; i < NI; i += NTC) {
            const int x = i % NB, y = (i / NB) % NB, z = NDIM == 3 ? i / (NB * NB) : 0;
            const int c = lin<NDIM>(x, y, z);
            U[e0 + c] = S[e0 + c];
        }
    }
}

#define COND_DISPATCH(ndim, fp64, KER, ...)                                \
    do {                                                                   \
        if (ndim == 2) {                                                   \
            if (fp64)                                                      \
                hipLaunchKernelGGL((KER<2, double>), __VA_ARGS__);         \
            else                                                           \
                hipLaunchKernelGGL((KER<2, float>), __VA_ARGS__);          \
        } else {                                                           \
            if (fp64)                                                      \
                hipLaunchKernelGGL((KER<3, double>), __VA_ARGS__);         \
            else                                                           \
                hipLaunchKernelGGL((KER<3, float>), __VA_ARGS__);          \
        }                                                                  \
    } while (0)

template <int NDIM, typename T>
static void launch_conduct_t(const CondArgs &a, hipStream_t s)
{
    if (a.mode == MAP_COND_FIELD)
        hipLaunchKernelGGL((k_conduct<NDIM, T, MAP_COND_FIELD>), dim3(a.nitems), dim3(NTC), 0, s, a);
    else
        hipLaunchKernelGGL((k_conduct<NDIM, T, MAP_COND_ISO>), dim3(a.nitems), dim3(NTC), 0, s, a);
}

hipError_t launch_conduct(int ndim, bool fp64, const CondArgs &a, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    if (ndim == 2)
        fp64 ? launch_conduct_t<2, double>(a, s) : launch_conduct_t<2, float>(a, s);
    else
        fp64 ? launch_conduct_t<3, double>(a, s) : launch_conduct_t<3, float>(a, s);
    return hipGetLastError();
}

hipError_t launch_cond_commit(int ndim, bool fp64, const CondArgs &a, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    COND_DISPATCH(ndim, fp64, k_cond_commit, dim3(a.nitems), dim3(NTC), 0, s, a);
    return hipGetLastError();
}

}  // namespace mapk
