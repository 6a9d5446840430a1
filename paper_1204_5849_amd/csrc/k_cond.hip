// k_cond.hip -- one sub-step of the thermal-conduction subcycle (paper
// Sec. 3.4): the energy alone advances by the explicit conduction scheme,
// isotropic or along the magnetic field, with the other variables frozen.
//
// Three launches per sub-step, around the energy-only boundary passes:
//   * prep: T = p / rho and kappa = kappa0 T^n at every cell a reader can
//     reach through the ghost descriptors (the interiors of all blocks, and
//     the ghost cells of leaves that hold their own prolongated values),
//     into planes 0 and 1 of the workspace's shadow state (free between
//     steps; same tile layout as U, so a descriptor offset addresses both);
//   * conduct: per leaf cell, the energy fluxes through its faces from T,
//     kappa and B read where the descriptors point, the new energy into the
//     shadow's energy plane, and the fluxes of faces shared with another
//     level into the reflux buffer;
//   * commit: the new energy of every leaf cell back into U (a separate
//     pass, since conduct reads neighbours' old values).
// Arithmetic is FP64 for both state precisions and follows the written
// order (no contraction): the conduction passes are gathers, not ALU-bound.
#include "kernels.hpp"
#include "physics.hpp"
#include "tile.hpp"

#pragma clang fp contract(off)

namespace mapk {

namespace {
constexpr int NTC = 256;
}

template <int NDIM, typename T>
__global__ void __launch_bounds__(NTC) k_cond_prep(CondArgs a)
{
    constexpr int P = tile_cells<NDIM>();
    const T *U = (const T *)a.U;
    T *S = (T *)a.S;
    const double gm1 = a.gamma - 1.0;
    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const int slot = a.list ? a.list[item] : item;
        const BlockRec br = a.blk[slot];
        if (a.sub >= a.dt[br.sim].nsub)
            continue;
        const size_t base = (size_t)slot * NV * P;
        for (int c = threadIdx.x; c < P; c += NTC) {
            const int x = c % PD - NG, y = (c / PD) % PD - NG;
            const int z = NDIM == 3 ? c / (PD * PD) - NG : 0;
            const bool inside = x >= 0 && x < NB && y >= 0 && y < NB &&
                                (NDIM == 2 || (z >= 0 && z < NB));
            if (!inside && (!br.leaf || cell_src<NDIM>(a.desc, slot, x, y, z) != base + c))
                continue;
            double u[EN + 1];
#pragma unroll
            for (int k = 0; k <= EN; k++)
                u[k] = (double)U[base + (size_t)k * P + c];
            const double ir = 1.0 / u[RHO];
            const double vx = u[MX] * ir, vy = u[MY] * ir, vz = u[MZ] * ir;
            const double ke = 0.5 * (u[MX] * vx + u[MY] * vy + u[MZ] * vz);
            const double me = 0.5 * (u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ]);
            const double pr = gm1 * (u[EN] - ke - me);
            const double Tt = pr / u[RHO];
            S[base + c] = (T)Tt;
            S[base + P + c] = (T)kappa_of(a.kappa0, a.khalf, Tt);
        }
    }
}

// energy flux along +d through the face between the cell at (x, y, z) and
// its +d neighbour, F = -(kappa grad T)_d: the face kappa is the geometric
// mean of the two cells'; isotropic, F = -kappa_f (T_n - T_c)/dx_d; along the
// field, F = -kappa_f b_d (b . grad T) with b from the mean of the two cells'
// fields and grad T at the face: the difference across it along d, and along
// each other dimension the mean of the two cells' central differences (zero
// where the face field vanishes)
template <int NDIM, typename T, int MODE>
__device__ __forceinline__ double cond_flux(const CondArgs &a, const T *U, const T *S, int slot,
                                            int d, int x, int y, int z, const double *dxp)
{
    constexpr int P = tile_cells<NDIM>();
    auto off = [&](int xx, int yy, int zz) { return cell_src<NDIM>(a.desc, slot, xx, yy, zz); };
    const int nx = x + (d == 0), ny = y + (d == 1), nz = z + (d == 2);
    const size_t oc = off(x, y, z), on = off(nx, ny, nz);
    const double kf = sqrt((double)S[oc + P] * (double)S[on + P]);
    const double gd = ((double)S[on] - (double)S[oc]) / dxp[d];
    if constexpr (MODE == MAP_COND_ISO) {
        return -(kf * gd);
    } else {
        double Bf[3], bb = 0.0;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            Bf[j] = 0.5 * ((double)U[oc + (size_t)(BX + j) * P] + (double)U[on + (size_t)(BX + j) * P]);
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
            } else if (e < NDIM) {
                const int ex = e == 0, ey = e == 1, ez = e == 2;
                const double tcp = (double)S[off(x + ex, y + ey, z + ez)];
                const double tcm = (double)S[off(x - ex, y - ey, z - ez)];
                const double tnp = (double)S[off(nx + ex, ny + ey, nz + ez)];
                const double tnm = (double)S[off(nx - ex, ny - ey, nz - ez)];
                g = ((tcp - tcm) + (tnp - tnm)) / (4.0 * dxp[e]);
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
    constexpr int NI = NDIM == 3 ? NB * NB * NB : NB * NB;
    constexpr int FC = NDIM == 3 ? NB * NB : NB;
    const T *U = (const T *)a.U;
    T *S = (T *)a.S;
    T *fbuf = (T *)a.fbuf;
    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const int slot = a.list[item];
        const BlockRec br = a.blk[slot];
        const map_dt rec = a.dt[br.sim];
        if (a.sub >= rec.nsub)
            continue;
        const double *dxp = a.lvl_dx + ((size_t)br.sim * (MAXL + 1) + br.level) * 3;
        const size_t base = (size_t)slot * NV * P;
        for (int i = threadIdx.x; i < NI; i += NTC) {
            const int x = i % NB, y = (i / NB) % NB, z = NDIM == 3 ? i / (NB * NB) : 0;
            const int q[3] = {x, y, z};
            double acc = 0.0;
#pragma unroll
            for (int d = 0; d < NDIM; d++) {
                const double fp = cond_flux<NDIM, T, MODE>(a, U, S, slot, d, x, y, z, dxp);
                const double fm = cond_flux<NDIM, T, MODE>(a, U, S, slot, d, x - (d == 0),
                                                           y - (d == 1), z - (d == 2), dxp);
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

hipError_t launch_cond_prep(int ndim, bool fp64, const CondArgs &a, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    COND_DISPATCH(ndim, fp64, k_cond_prep, dim3(a.nitems), dim3(NTC), 0, s, a);
    return hipGetLastError();
}

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
