// k_cond.hip -- one sub-step of the thermal-conduction subcycle (paper
// Sec. 3.4): the energy alone advances by the explicit conduction scheme,
// isotropic or along the magnetic field, with the other variables frozen.
//
// Two launches per sub-step, around the energy-only boundary passes:
//   * conduct: one workgroup of five waves per leaf marches along z (3-D)
//     with a window of four 18 x 18 planes in LDS (the interior and the first
//     ring of ghost cells, edges and corners included): each plane is
//     gathered where the ghost descriptors point, and its T = p / rho,
//     sqrt(kappa), kappa = kappa0 T^n, and along the field B, are formed once
//     per cell.  Every face flux is then evaluated once: the 17 x 16 x-faces
//     and 16 x 17 y-faces of the plane by one thread each into LDS, the face
//     above each interior cell by that cell's thread, which keeps it for the
//     next plane.  The new energy goes to the energy plane of a scratch state
//     (the update reads neighbours' old values), the fluxes of faces shared
//     with another level to the reflux buffer;
//   * commit: the new energy of every leaf cell back into U.
// Arithmetic is FP64 for both state precisions and follows the written
// order (no contraction); divisions by the cell size are multiplications by
// its reciprocal, formed once per block.
#include "kernels.hpp"
#include "physics.hpp"
#include "tile.hpp"

#pragma clang fp contract(off)

namespace mapk {

namespace {
constexpr int NTC = 256;         // commit
constexpr int NTK = 320;         // conduct: five waves, one per x- or y-face of a plane
constexpr int RW = NB + 2;       // ring width: cells -1 .. NB
constexpr int RP = RW * RW;      // cells of one window plane
constexpr int NWIN = 4;          // window planes (z-1, z, z+1 and the one being loaded)
constexpr int NF = (NB + 1) * NB;  // x-faces (or y-faces) of one plane
static_assert(NF <= NTK && NB * NB <= NTK && RP <= 2 * NTK, "conduct lane layout");
}  // namespace

// one window plane: T, sqrt(kappa), the energy and (along the field) the
// field of the cells (x, y) in [-1, NB]^2 at one z; energy and field keep the
// state's precision (exact), so that the FP32 kernel fits three workgroups
// per CU
template <int MODE, typename BT>
struct CondPlane {
    double T[RP], S[RP];
    BT E[RP];
    BT B[MODE == MAP_COND_FIELD ? 3 : 1][MODE == MAP_COND_FIELD ? RP : 1];
};

// the variables rho .. e of the cell at offset o (variable 0)
template <int NDIM, typename T>
__device__ __forceinline__ void cond_load(const T *U, size_t o, T (&r)[EN + 1])
{
    constexpr int P = tile_cells<NDIM>();
#pragma unroll
    for (int k = 0; k <= EN; k++)
        r[k] = U[o + (size_t)k * P];
}

// window cell i of a plane from its variables r
template <typename T, int MODE>
__device__ __forceinline__ void cond_form(const CondArgs &a, const T (&r)[EN + 1], int i,
                                          CondPlane<MODE, T> &pl, double gm1)
{
    double u[EN + 1];
#pragma unroll
    for (int k = 0; k <= EN; k++)
        u[k] = (double)r[k];
    {
        const double ir = 1.0 / u[RHO];
        const double vx = u[MX] * ir, vy = u[MY] * ir, vz = u[MZ] * ir;
        const double ke = 0.5 * (u[MX] * vx + u[MY] * vy + u[MZ] * vz);
        const double me = 0.5 * (u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ]);
        const double Tt = gm1 * (u[EN] - ke - me) / u[RHO];
        pl.T[i] = Tt;
        pl.S[i] = sqrt(kappa_of(a.kappa0, a.khalf, Tt));
        pl.E[i] = r[EN];
        if constexpr (MODE == MAP_COND_FIELD) {
            pl.B[0][i] = (T)u[BX];
            pl.B[1][i] = (T)u[BY];
            pl.B[2][i] = (T)u[BZ];
        }
    }
}

// energy flux along +d through the face between cell c (index ic of plane
// pc) and its +d neighbour (index in of plane pn), F = -(kappa grad T)_d:
// the face kappa is the geometric mean of the two cells', sqrt(kappa_c)
// sqrt(kappa_n); isotropic, F = -kappa_f (T_n - T_c)/dx_d; along the field,
// F = -kappa_f b_d (b . grad T) with b from the mean of the two cells' fields
// and grad T at the face: the difference across it along d, and along each
// other dimension e the mean of the two cells' central differences (planes
// pcm/pcp and pnm/pnp hold the z neighbours of c and n; zero where the face
// field vanishes).  idx = 1/dx per dimension.
template <int NDIM, int MODE, typename PL>
__device__ __forceinline__ double face_flux_c(const PL *pc, int ic, const PL *pn, int in, int d,
                                              const PL *pcm, const PL *pcp, const PL *pnm,
                                              const PL *pnp, const double *idx)
{
    const double kf = pc->S[ic] * pn->S[in];
    const double gd = (pn->T[in] - pc->T[ic]) * idx[d];
    if constexpr (MODE == MAP_COND_ISO) {
        return -(kf * gd);
    } else {
        double Bf[3], bb = 0.0;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            Bf[j] = 0.5 * ((double)pc->B[j][ic] + (double)pn->B[j][in]);
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
                g = ((pcp->T[ic] - pcm->T[ic]) + (pnp->T[in] - pnm->T[in])) * (0.25 * idx[e]);
            } else if (e < 2) {
                const int s = e == 0 ? 1 : RW;
                g = ((pc->T[ic + s] - pc->T[ic - s]) + (pn->T[in + s] - pn->T[in - s])) *
                    (0.25 * idx[e]);
            } else {
                g = 0.0;
            }
            bg += Bf[e] * g;
        }
        return -(kf * Bf[d] * bg / bb);
    }
}

template <int NDIM, typename T, int MODE>
__global__ void __launch_bounds__(NTK) k_conduct(CondArgs a)
{
    constexpr int P = tile_cells<NDIM>();
    constexpr int XS = PD * PD;  // z stride of a padded 3-D tile
    constexpr int FC = NDIM == 3 ? NB * NB : NB;
    constexpr int NW = NDIM == 3 ? NWIN : 1;
    using Plane = CondPlane<MODE, T>;
    __shared__ Plane win[NW];
    __shared__ double fx[2][NF], fy[2][NF];  // x- and y-face fluxes of a plane (by parity)
    const T *U = (const T *)a.U;
    T *S = (T *)a.S;
    T *fbuf = (T *)a.fbuf;
    const double gm1 = a.gamma - 1.0;
    const int t = threadIdx.x;
    const bool iscell = t < NB * NB;
    const int qx = t % NB, qy = t / NB;  // this thread's interior column
    const int ic0 = (qy + 1) * RW + qx + 1;
    // this thread's x-face (between x = fxx - 1 and fxx in row fxy) and
    // y-face (between y = fyy - 1 and fyy in column fyx)
    const bool isface = t < NF;
    const int fxx = t % (NB + 1), fxy = t / (NB + 1);
    const int fyx = t % NB, fyy = t / NB;
    // this thread's window cells: t and t + NTK
    const bool g2 = t + NTK < RP;
    const int gx0 = t % RW - 1, gy0 = t / RW - 1;
    const int gx1 = (t + NTK) % RW - 1, gy1 = (t + NTK) / RW - 1;
    if (sub_idle(a.dt, a.nsims, a.sub))
        return;
    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const int slot = a.list[item];
        const BlockRec br = a.blk[slot];
        const map_dt rec = a.dt[br.sim];
        if (a.sub >= rec.nsub)
            continue;
        const double *dxp = a.lvl_dx + ((size_t)br.sim * (MAXL + 1) + br.level) * 3;
        const double idx[3] = {1.0 / dxp[0], 1.0 / dxp[1], 1.0 / dxp[2]};
        const size_t base = (size_t)slot * NV * P;
        int fbs[6];
#pragma unroll
        for (int k = 0; k < 6; k++)
            fbs[k] = a.fbidx[(size_t)slot * 6 + k];
        // reflux buffer entry of the face of side `side` along d at in-face
        // position (i, j), or -1
        auto fb_at = [&](int d, int side, int i, int j) -> long {
            const int fb = side ? fbs[2 * d + 1] : fbs[2 * d];
            return fb < 0 ? -1 : ((long)fb * NV + EN) * FC + i + NB * j;
        };
        // x- and y-faces of plane z (planes zm / zp: its z neighbours) into
        // buffer b
        auto inplane_faces = [&](int z, const Plane *pm, const Plane *p0, const Plane *pp, int b) {
            if (!isface)
                return;
            {
                const int ic = (fxy + 1) * RW + fxx;
                const double f = face_flux_c<NDIM, MODE>(p0, ic, p0, ic + 1, 0, pm, pp, pm, pp, idx);
                fx[b][t] = f;
                if (fxx == 0 || fxx == NB) {
                    const long e = fb_at(0, fxx == NB, fxy, z);
                    if (e >= 0)
                        fbuf[e] = (T)f;
                }
            }
            {
                const int ic = fyy * RW + fyx + 1;
                const double f = face_flux_c<NDIM, MODE>(p0, ic, p0, ic + RW, 1, pm, pp, pm, pp, idx);
                fy[b][t] = f;
                if (fyy == 0 || fyy == NB) {
                    const long e = fb_at(1, fyy == NB, fyx, z);
                    if (e >= 0)
                        fbuf[e] = (T)f;
                }
            }
        };
        // update of this thread's cell of plane z (window plane pl) from
        // buffer b and the z fluxes below and above
        auto update = [&](int z, const Plane *pl, int b, double fzm, double fzp) {
            const double e = (double)pl->E[ic0];
            double acc = (fx[b][qy * (NB + 1) + qx + 1] - fx[b][qy * (NB + 1) + qx]) * idx[0];
            acc += (fy[b][(qy + 1) * NB + qx] - fy[b][qy * NB + qx]) * idx[1];
            if constexpr (NDIM == 3)
                acc += (fzp - fzm) * idx[2];
            S[base + (size_t)EN * P + lin<NDIM>(qx, qy, z)] = (T)(e - rec.dt_sub * acc);
        };
        if constexpr (NDIM == 2) {
            T r[EN + 1];
            cond_load<2, T>(U, cell_src<2>(a.desc, slot, gx0, gy0, 0), r);
            cond_form<T, MODE>(a, r, t, win[0], gm1);
            if (g2) {
                cond_load<2, T>(U, cell_src<2>(a.desc, slot, gx1, gy1, 0), r);
                cond_form<T, MODE>(a, r, t + NTK, win[0], gm1);
            }
            __syncthreads();
            inplane_faces(0, &win[0], &win[0], &win[0], 0);
            __syncthreads();
            if (iscell)
                update(0, &win[0], 0, 0.0, 0.0);
            __syncthreads();
        } else {
            // sources of this thread's window cells below the block, in its
            // z range (one region, linear in z) and above it
            const size_t o0[3] = {cell_src<3>(a.desc, slot, gx0, gy0, -1),
                                  cell_src<3>(a.desc, slot, gx0, gy0, 0),
                                  cell_src<3>(a.desc, slot, gx0, gy0, NB)};
            // (threads with one window cell read it twice, so that every
            // thread has the same loads in flight and the waits stay exact)
            size_t o1[3] = {o0[0], o0[1], o0[2]};
            if (g2) {
                o1[0] = cell_src<3>(a.desc, slot, gx1, gy1, -1);
                o1[1] = cell_src<3>(a.desc, slot, gx1, gy1, 0);
                o1[2] = cell_src<3>(a.desc, slot, gx1, gy1, NB);
            }
            auto at = [&](const size_t (&o)[3], int z) {
                return z < 0 ? o[0] : (z < NB ? o[1] + (size_t)z * XS : o[2]);
            };
            // window slot of plane p: (p + 1) mod 4; planes -1 .. NB
            auto W = [&](int p) { return &win[(p + 1) & (NWIN - 1)]; };
            // a plane's window cells go through registers: their loads are
            // issued one plane before they are formed into the window
            T r0[EN + 1], r1[EN + 1];
            auto issue = [&](int z) {
                cond_load<3, T>(U, at(o0, z), r0);
                cond_load<3, T>(U, at(o1, z), r1);
            };
            auto form = [&](int z) {
                cond_form<T, MODE>(a, r0, t, *W(z), gm1);
                if (g2)
                    cond_form<T, MODE>(a, r1, t + NTK, *W(z), gm1);
            };
            for (int p = -1; p <= 1; p++) {
                issue(p);
                form(p);
            }
            issue(2);
            __syncthreads();
            // the face z = -1/2 below each column
            double fzm = 0.0;
            if (iscell) {
                fzm = face_flux_c<3, MODE>(W(-1), ic0, W(0), ic0, 2, W(-1), W(-1), W(0), W(0), idx);
                const long e = fb_at(2, 0, qx, qy);
                if (e >= 0)
                    fbuf[e] = (T)fzm;
            }
            for (int z = 0; z < NB; z++) {
                // plane z+2 (requested one plane ago) goes into the slot
                // plane z-2 left, and plane z+3 is requested, while the faces
                // of plane z are formed from z-1, z and z+1
                if (z + 2 <= NB)
                    form(z + 2);
                if (z + 3 <= NB)
                    issue(z + 3);
                inplane_faces(z, W(z - 1), W(z), W(z + 1), z & 1);
                double fzp = 0.0;
                if (iscell) {
                    // z faces: the transverse gradients are in-plane
                    fzp = face_flux_c<3, MODE>(W(z), ic0, W(z + 1), ic0, 2, W(z), W(z), W(z + 1),
                                               W(z + 1), idx);
                    if (z == NB - 1) {
                        const long e2 = fb_at(2, 1, qx, qy);
                        if (e2 >= 0)
                            fbuf[e2] = (T)fzp;
                    }
                }
                // one barrier per plane: the face buffers alternate, and the
                // slot the next gather overwrites was last read before it
                __syncthreads();
                if (iscell)
                    update(z, W(z), z & 1, fzm, fzp);
                fzm = fzp;
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
    if (sub_idle(a.dt, a.nsims, a.sub))
        return;
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

// (k_conduct keeps one workgroup per leaf: its occupancy is set by LDS, and
// a persistent grid of SUB_GRID workgroups ended on a partial round and ran
// 9 % slower; an idle one returns after one read)
static int sub_grid(const CondArgs &a) { return a.nitems > SUB_GRID ? SUB_GRID : a.nitems; }

template <int NDIM, typename T>
static void launch_conduct_t(const CondArgs &a, hipStream_t s)
{
    if (a.mode == MAP_COND_FIELD)
        hipLaunchKernelGGL((k_conduct<NDIM, T, MAP_COND_FIELD>), dim3(a.nitems), dim3(NTK), 0, s, a);
    else
        hipLaunchKernelGGL((k_conduct<NDIM, T, MAP_COND_ISO>), dim3(a.nitems), dim3(NTK), 0, s, a);
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
    COND_DISPATCH(ndim, fp64, k_cond_commit, dim3(sub_grid(a)), dim3(NTC), 0, s, a);
    return hipGetLastError();
}

}  // namespace mapk
