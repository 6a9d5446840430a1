// k_aux.hip -- the data-motion and reduction stages around the block update:
// ghost copies with periodic / outflow edges, conservative prolongation,
// restriction, reflux (paper Sec. 4.3), the CFL reduction and time-step record
// (Sec. 2, Sec. 3.7), FP64 totals and the primitive-to-conserved conversion.
//
// These kernels are HBM-bound gathers and scatters: threads walk the ghost
// frame (or interior) of a block in the padded tile's own linear order so
// that writes are contiguous rows, and each thread moves all nine variables
// of its cell.  Contraction of a*b+c into FMA is switched off here so the
// arithmetic follows the written order exactly (it costs nothing in a
// memory-bound kernel).
#include "cfl.hpp"
#include "kernels.hpp"
#include "physics.hpp"
#include "sched.hpp"
#include "tile.hpp"

#pragma clang fp contract(off)

namespace mapk {

template <int NDIM>
struct FG;
template <>
struct FG<2> {
    static constexpr int P = PD * PD, NGC = PD * PD - NB * NB, BPW = 16, NI = NB * NB;
};
template <>
struct FG<3> {
    static constexpr int P = PD * PD * PD, NGC = PD * PD * PD - NB * NB * NB, BPW = 1,
                         NI = NB * NB * NB;
};
constexpr int NTA = 256;

// two adjacent values along x (8- or 16-byte aligned at even padded indices)
template <typename T>
struct Pair;
template <>
struct Pair<float> {
    using V = float2;
};
template <>
struct Pair<double> {
    using V = double2;
};

// g-th ghost cell of a block, enumerated in the padded tile's linear order
// by regions: the ghost planes/rows below and above, then the side strips
template <int NDIM>
__device__ __forceinline__ void ghost_xyz(int g, int &x, int &y, int &z)
{
    if constexpr (NDIM == 2) {
        z = 0;
        if (g < 4 * PD) {
            int r = g / PD;
            x = g - r * PD - NG;
            y = r < 2 ? r - 2 : r + NB - 2;
        } else {
            g -= 4 * PD;
            int r = g >> 2, c = g & 3;
            y = r;
            x = c < 2 ? c - 2 : c + NB - 2;
        }
    } else {
        if (g < 4 * PD * PD) {
            int pl = g / (PD * PD), r = g - pl * PD * PD;
            z = pl < 2 ? pl - 2 : pl + NB - 2;
            y = r / PD - NG;
            x = r % PD - NG;
        } else if (g < 4 * PD * PD + NB * 4 * PD) {
            g -= 4 * PD * PD;
            z = g / (4 * PD);
            int r = g - z * 4 * PD, row = r / PD;
            y = row < 2 ? row - 2 : row + NB - 2;
            x = r % PD - NG;
        } else {
            g -= 4 * PD * PD + NB * 4 * PD;
            z = g / (NB * 4);
            int r = g - z * NB * 4;
            y = r >> 2;
            int c = r & 3;
            x = c < 2 ? c - 2 : c + NB - 2;
        }
    }
}

// variables a pass moves: all, or the energy alone (EO, conduction sub-steps)
template <bool EO>
struct VarRange {
    static constexpr int K0 = EO ? EN : 0, K1 = EO ? EN + 1 : NV;
};

// a conduction sub-step pass skips the blocks of simulations whose subcycle
// has fewer sub-steps
__device__ __forceinline__ bool sub_inactive(const map_dt *dt, int sim, int sub)
{
    return sub >= dt[sim].nsub;
}

// ---- same-level copies and physical edges (descriptor src >= 0)
template <int NDIM, typename T, bool EO>
__global__ void __launch_bounds__(NTA) k_fill_copy(FillArgs a)
{
    constexpr int P = FG<NDIM>::P, NGC = FG<NDIM>::NGC, BPW = FG<NDIM>::BPW;
    constexpr int K0 = VarRange<EO>::K0, K1 = VarRange<EO>::K1;
    T *U = (T *)a.U;
    if (EO && sub_idle(a.dt, a.nsims, a.sub))
        return;
    int first, stride, end;
    xcd_range(a.nitems, first, stride, end);
    for (int item = first; item < end; item += stride) {
        // one block per item (3-D): its selection is loaded once
        FrameSel f1{~0u, {-NG, -NG, -NG}, {NB + NG - 1, NB + NG - 1, NB + NG - 1}, 0};
        if (BPW == 1 && a.copy_sel && a.slot_base + item < a.slot_end)
            f1 = a.copy_sel[a.slot_base + item];
        for (int g = threadIdx.x; g < BPW * NGC; g += NTA) {
            const int lb = g / NGC, gi = g - lb * NGC;
            const int i = a.slot_base + item * BPW + lb;
            if (i >= a.slot_end)
                break;
            const int slot = a.copy_list ? a.copy_list[i] : i;
            if (EO && sub_inactive(a.dt, a.blk[slot].sim, a.sub))
                continue;
            int x, y, z;
            ghost_xyz<NDIM>(gi, x, y, z);
            const int di = dir_index<NDIM>(x, y, z);
            if (BPW == 1 || a.copy_sel) {
                const FrameSel &f = BPW == 1 ? f1 : a.copy_sel[i];
                if (!((f.dirs >> di) & 1u) || x < f.lo[0] || x > f.hi[0] || y < f.lo[1] ||
                    y > f.hi[1] || (NDIM == 3 && (z < f.lo[2] || z > f.hi[2])))
                    continue;
            }
            const Desc ds = a.desc[(size_t)slot * NDIR + di];
            if (ds.src < 0)
                continue;
            const int sx = src_index(x, ds.o0), sy = src_index(y, ds.o1);
            const int sz = NDIM == 3 ? src_index(z, ds.o2) : 0;
            T *dst = U + (size_t)slot * NV * P + lin<NDIM>(x, y, z);
            const T *src = U + (size_t)ds.src * NV * P + lin<NDIM>(sx, sy, sz);
            T v[NV];
#pragma unroll
            for (int k = K0; k < K1; k++)
                v[k] = src[(size_t)k * P];
#pragma unroll
            for (int k = K0; k < K1; k++)
                dst[(size_t)k * P] = v[k];
        }
    }
}

// minmod-limited linear interpolation from the parent's padded tile at fine
// padded cell (x, y, z) of a child in position cpos (Sec. 4.3, step 6)
template <int NDIM, typename T, int K0 = 0, int K1 = NV>
__device__ __forceinline__ void prolong_cell(const T *pu, int cpos, int x, int y, int z, T out[NV])
{
    constexpr int P = FG<NDIM>::P;
    const int loc[3] = {x, y, z};
    int ci[3] = {0, 0, 0};
    T w[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < NDIM; d++) {
        int f = ((cpos >> d) & 1) * NB + loc[d];
        ci[d] = f >> 1;  // floor(f / 2), also for f < 0
        w[d] = (f & 1) ? T(0.25) : T(-0.25);
    }
    const int c = lin<NDIM>(ci[0], ci[1], ci[2]);
    const int st[3] = {1, PD, PD * PD};
#pragma unroll
    for (int k = K0; k < K1; k++) {
        const T *q = pu + (size_t)k * P;
        T val = q[c];
        T v = val;
#pragma unroll
        for (int d = 0; d < NDIM; d++) {
            T s = lim_minmod(q[c + st[d]] - val, val - q[c - st[d]]);
            v = v + s * w[d];
        }
        out[k] = v;
    }
}

// ---- prolongated ghosts of the blocks of one level (descriptor src == -1)
// Every ghost region of a child is a union of 2^d-cell groups whose fine
// cells lie in one parent cell: the group shares that cell's value and
// limited slopes, and its cells differ only in the signs of the quarter-
// slope terms.  One thread forms a whole group (the operations of
// prolong_cell, in its order, per fine cell) and stores it as x pairs.
// Groups are enumerated over the child's padded tile at parent resolution
// (10^d cells, the 8^d interior ones skipped): the planes below and above,
// then the rows, then the columns.
template <int NDIM>
__device__ __forceinline__ void group_xyz(int g, int &X, int &Y, int &Z)
{
    constexpr int H = NB / 2, Q = H + 2;  // interior and padded groups per dimension
    if constexpr (NDIM == 2) {
        Z = 0;
        if (g < 2 * Q) {
            const int r = g / Q;
            X = g - r * Q - 1;
            Y = r ? H : -1;
        } else {
            g -= 2 * Q;
            Y = g >> 1;
            X = (g & 1) ? H : -1;
        }
    } else {
        if (g < 2 * Q * Q) {
            const int pl = g / (Q * Q), r = g - pl * Q * Q;
            Z = pl ? H : -1;
            Y = r / Q - 1;
            X = r % Q - 1;
        } else if (g < 2 * Q * Q + H * 2 * Q) {
            g -= 2 * Q * Q;
            Z = g / (2 * Q);
            const int r = g - Z * 2 * Q;
            Y = r < Q ? -1 : H;
            X = r % Q - 1;
        } else {
            g -= 2 * Q * Q + H * 2 * Q;
            Z = g / (2 * H);
            const int r = g - Z * 2 * H;
            Y = r >> 1;
            X = (r & 1) ? H : -1;
        }
    }
}

template <int NDIM, typename T, bool EO>
__global__ void __launch_bounds__(NTA) k_prolong_ghosts(FillArgs a)
{
    using V = typename Pair<T>::V;
    constexpr int P = FG<NDIM>::P, H = NB / 2, Q = H + 2;
    constexpr int NGG = NDIM == 3 ? Q * Q * Q - H * H * H : Q * Q - H * H;  // ghost groups
    constexpr int K0 = VarRange<EO>::K0, K1 = VarRange<EO>::K1;
    T *U = (T *)a.U;
    if (EO && sub_idle(a.dt, a.nsims, a.sub))
        return;
    int first, stride, end;
    xcd_range(a.nitems, first, stride, end);  // siblings share the parent tile in L2
    for (int item = first; item < end; item += stride) {
        const int slot = a.list[item];
        if (EO && sub_inactive(a.dt, a.blk[slot].sim, a.sub))
            continue;
        const int par = a.parent[slot];
        const int cpos = a.blk[slot].cpos;
        const T *pu = U + (size_t)par * NV * P;
        T *ub = U + (size_t)slot * NV * P;
        // the directions whose descriptor has no source, loaded once per block
        const uint32_t pm = a.list_mask[item];
        for (int g = threadIdx.x; g < NGG; g += NTA) {
            int X, Y, Z;
            group_xyz<NDIM>(g, X, Y, Z);
            const int x = 2 * X, y = 2 * Y, z = NDIM == 3 ? 2 * Z : 0;
            if (!((pm >> dir_index<NDIM>(x, y, z)) & 1u))
                continue;
            // the parent cell of the group
            const int c = lin<NDIM>((cpos & 1) * H + X, ((cpos >> 1) & 1) * H + Y,
                                    NDIM == 3 ? ((cpos >> 2) & 1) * H + Z : 0);
            const int st[3] = {1, PD, PD * PD};
            const int f0 = lin<NDIM>(x, y, z);
#pragma unroll
            for (int k = K0; k < K1; k++) {
                const T *q = pu + (size_t)k * P;
                const T val = q[c];
                T sw[3];  // quarter slope along each dimension
#pragma unroll
                for (int d = 0; d < NDIM; d++)
                    sw[d] = lim_minmod(q[c + st[d]] - val, val - q[c - st[d]]) * T(0.25);
                T *o = ub + (size_t)k * P + f0;
#pragma unroll
                for (int j = 0; j < (NDIM == 3 ? 4 : 2); j++) {
                    const int jy = j & 1, jz = j >> 1;  // fine cell 2Y + jy, 2Z + jz
                    // v = ((val + s0 w0) + s1 w1) + s2 w2 with w = -1/4 (even
                    // fine index) or +1/4 (odd); -s/4 is exact
                    T lo = val - sw[0], hi = val + sw[0];
                    const T ty = jy ? sw[1] : -sw[1];
                    lo = lo + ty;
                    hi = hi + ty;
                    if constexpr (NDIM == 3) {
                        const T tz = jz ? sw[2] : -sw[2];
                        lo = lo + tz;
                        hi = hi + tz;
                    }
                    V pr;
                    pr.x = lo;
                    pr.y = hi;
                    *reinterpret_cast<V *>(o + jy * PD + (NDIM == 3 ? jz * PD * PD : 0)) = pr;
                }
            }
        }
    }
}

// ---- whole-block prolongation (regrid initialisation)
template <int NDIM, typename T>
__global__ void __launch_bounds__(NTA) k_prolong_blocks(FillArgs a)
{
    constexpr int P = FG<NDIM>::P, NI = FG<NDIM>::NI;
    T *U = (T *)a.U;
    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const int slot = a.list[item];
        const int par = a.parent[slot];
        if (par < 0)
            continue;
        const int cpos = a.blk[slot].cpos;
        const T *pu = U + (size_t)par * NV * P;
        T *ub = U + (size_t)slot * NV * P;
        for (int i = threadIdx.x; i < NI; i += NTA) {
            const int x = i % NB, y = (i / NB) % NB, z = NDIM == 3 ? i / (NB * NB) : 0;
            T v[NV];
            prolong_cell<NDIM, T>(pu, cpos, x, y, z, v);
            const int c = lin<NDIM>(x, y, z);
#pragma unroll
            for (int k = 0; k < NV; k++)
                ub[(size_t)k * P + c] = v[k];
        }
    }
}

// ---- restriction: parent interior = mean of the 2^d child cells it covers
// (Sec. 4.2, Sec. 4.3 step 1).  The two cells of an x pair are adjacent and
// 2-element aligned in the padded tile, so each pair is one vector load; the
// sum is taken x pairs first, then y, then z.

// The restriction kernel: one workgroup per parent, one parent cell per
// thread and pass, or, for a level with fewer parents than CUs, one
// workgroup per child (the parent's octant it covers; the same sums).  With
// CFL it also forms the CFL maxima of the leaf
// children (the values it reads are the leaves' final ones after reflux),
// so that the next cycle's dt needs no pass of its own over those leaves: a
// thread's parent cells lie in one child per half of the parent in z, each
// thread keeps its maxima per half, and the workgroup combines them per
// child with LDS atomics on the bit patterns (the speeds are finite and
// non-negative, so those order like the values).
template <int NDIM, typename T, bool EO, bool CFL = false>
__global__ void __launch_bounds__(NTA) k_restrict(RestrictArgs a)
{
    using V = typename Pair<T>::V;
    constexpr int P = FG<NDIM>::P, NI = FG<NDIM>::NI;
    constexpr int K0 = VarRange<EO>::K0, K1 = VarRange<EO>::K1;
    constexpr int NCH = NDIM == 3 ? 8 : 4, NC = NDIM == 3 ? 8 : 4;
    constexpr int H = NB / 2, NO = NDIM == 3 ? H * H * H : H * H;  // parent cells per child
    static_assert(!CFL || (!EO && NTA == NB * NB), "CFL: all variables, one column per thread");
    __shared__ unsigned long long smax[CFL ? NCH : 1];
    __shared__ double red[CFL ? NTA / 64 : 1];
    T *U = (T *)a.U;
    if (EO && sub_idle(a.dt, a.nsims, a.sub))
        return;
    // parent cell d of ub from the 2^d cells of child tile cu at c0 (its
    // lowest corner), keeping those cells' values in cv for the CFL speeds
    auto restrict_cell = [&](T *ub, const T *cu, int c0, int d, T (&cv)[CFL ? NV : 1][CFL ? NC : 1]) {
#pragma unroll
        for (int k = K0; k < K1; k++) {
            const T *q = cu + (size_t)k * P + c0;
            const V r0 = *reinterpret_cast<const V *>(q);
            const V r1 = *reinterpret_cast<const V *>(q + PD);
            T v;
            if constexpr (NDIM == 2) {
                v = ((r0.x + r0.y) + (r1.x + r1.y)) * T(0.25);
            } else {
                const V r2 = *reinterpret_cast<const V *>(q + PD * PD);
                const V r3 = *reinterpret_cast<const V *>(q + PD * PD + PD);
                v = (((r0.x + r0.y) + (r1.x + r1.y)) + ((r2.x + r2.y) + (r3.x + r3.y))) * T(0.125);
                if constexpr (CFL) {
                    cv[k][4] = r2.x;
                    cv[k][5] = r2.y;
                    cv[k][6] = r3.x;
                    cv[k][7] = r3.y;
                }
            }
            if constexpr (CFL) {
                cv[k][0] = r0.x;
                cv[k][1] = r0.y;
                cv[k][2] = r1.x;
                cv[k][3] = r1.y;
            }
            ub[(size_t)k * P + d] = v;
        }
    };
    // the CFL speeds of those child cells into the running maximum mh
    auto cell_speeds = [&](const T (&cv)[CFL ? NV : 1][CFL ? NC : 1], double &mh, unsigned &bad,
                           unsigned &nonfin) {
        if constexpr (CFL) {
#pragma unroll
            for (int c = 0; c < NC; c++) {
                double u[NV];
                bool fin = true;
#pragma unroll
                for (int k = 0; k < NV; k++) {
                    u[k] = (double)cv[k][c];
                    fin = fin && isfinite(u[k]);
                }
                if (!fin) {
                    nonfin++;
                    continue;
                }
                double pr;
                bool b;
                const double sp = cfl_speed<NDIM>(u, a.gamma, pr, b);
                if (b)
                    bad++;
                mh = sp > mh ? sp : mh;
            }
        }
    };
    auto count = [&](unsigned bad, unsigned nonfin) {
        if (bad)
            atomicAdd(&a.cnt[2], (unsigned long long)bad);
        if (nonfin)
            atomicAdd(&a.cnt[3], (unsigned long long)nonfin);
    };
    if (a.per_child) {
        // one workgroup per child: the parent's octant (quadrant) it covers
        for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
            const int slot = a.list[item / NCH];
            const int cbit = item % NCH;
            if (EO && sub_inactive(a.dt, a.blk[slot].sim, a.sub))
                continue;
            T *ub = U + (size_t)slot * NV * P;
            const int child = a.children[(size_t)slot * 8 + cbit];
            const T *cu = U + (size_t)child * NV * P;
            const int ox = (cbit & 1) * H, oy = ((cbit >> 1) & 1) * H,
                      oz = NDIM == 3 ? ((cbit >> 2) & 1) * H : 0;
            const bool leafc = CFL && a.leaf_of[child] >= 0;
            double m = 0.0;
            unsigned bad = 0, nonfin = 0;
            for (int i = threadIdx.x; i < NO; i += NTA) {
                const int x = i % H, y = (i / H) % H, z = NDIM == 3 ? i / (H * H) : 0;
                T cv[CFL ? NV : 1][CFL ? NC : 1];
                restrict_cell(ub, cu, lin<NDIM>(2 * x, 2 * y, 2 * z), lin<NDIM>(ox + x, oy + y, oz + z),
                              cv);
                if (leafc)
                    cell_speeds(cv, m, bad, nonfin);
            }
            if constexpr (CFL) {
                count(bad, nonfin);
                // wave64 shuffle max, then across the waves through LDS
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double o = __shfl_xor(m, off, 64);
                    m = o > m ? o : m;
                }
                if ((threadIdx.x & 63) == 0)
                    red[threadIdx.x >> 6] = m;
                __syncthreads();
                if (threadIdx.x == 0 && leafc) {
                    double r = red[0];
                    for (int w = 1; w < NTA / 64; w++)
                        r = red[w] > r ? red[w] : r;
                    a.part[a.leaf_of[child]] = r;
                }
                __syncthreads();
            }
        }
        return;
    }
    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const int slot = a.list[item];
        if (EO && sub_inactive(a.dt, a.blk[slot].sim, a.sub))
            continue;
        T *ub = U + (size_t)slot * NV * P;
        double m[2] = {0.0, 0.0};
        unsigned bad = 0, nonfin = 0;
        if constexpr (CFL) {
            if (threadIdx.x < NCH)
                smax[threadIdx.x] = 0ull;
            __syncthreads();
        }
        for (int i = threadIdx.x; i < NI; i += NTA) {
            const int X = i % NB, Y = (i / NB) % NB, Z = NDIM == 3 ? i / (NB * NB) : 0;
            const int fx = 2 * X, fy = 2 * Y, fz = 2 * Z;
            const int cbit = (fx / NB) | ((fy / NB) << 1) | (NDIM == 3 ? (fz / NB) << 2 : 0);
            const int child = a.children[(size_t)slot * 8 + cbit];
            const T *cu = U + (size_t)child * NV * P;
            const int lx = fx % NB, ly = fy % NB, lz = NDIM == 3 ? fz % NB : 0;
            T cv[CFL ? NV : 1][CFL ? NC : 1];
            restrict_cell(ub, cu, lin<NDIM>(lx, ly, lz), lin<NDIM>(X, Y, Z), cv);
            if (CFL && a.leaf_of[child] >= 0)
                cell_speeds(cv, m[NDIM == 3 ? fz / NB : 0], bad, nonfin);
        }
        if constexpr (CFL) {
            // this thread's children: the one of its column below the middle
            // in z, and (3-D) the one above it
            const int cb = (threadIdx.x % NB >= NB / 2) | ((threadIdx.x / NB >= NB / 2) << 1);
            atomicMax(&smax[cb], (unsigned long long)__double_as_longlong(m[0]));
            if constexpr (NDIM == 3)
                atomicMax(&smax[cb | 4], (unsigned long long)__double_as_longlong(m[1]));
            count(bad, nonfin);
            __syncthreads();
            if (threadIdx.x < NCH) {
                const int li = a.leaf_of[a.children[(size_t)slot * 8 + threadIdx.x]];
                if (li >= 0)
                    a.part[li] = __longlong_as_double((long long)smax[threadIdx.x]);
            }
        }
    }
}

// ---- reflux: one workgroup per coarse leaf, its faces in a fixed order
template <int NDIM, typename T, bool EO>
__global__ void __launch_bounds__(NTA) k_reflux(RefluxArgs a)
{
    constexpr int P = FG<NDIM>::P;
    constexpr int FC = NDIM == 3 ? NB * NB : NB;
    constexpr int K0 = VarRange<EO>::K0, K1 = VarRange<EO>::K1;
    T *U = (T *)a.U;
    const T *fb = (const T *)a.fbuf;
    if (EO && sub_idle(a.dt, a.nsims, a.sub))
        return;
    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const int slot = a.slots[item];
        const BlockRec br = a.blk[slot];
        if (EO && sub_inactive(a.dt, br.sim, a.sub))
            continue;
        const double dtv = EO ? a.dt[br.sim].dt_sub : a.dt[br.sim].dt;
        const double *dxp = a.lvl_dx + ((size_t)br.sim * (MAXL + 1) + br.level) * 3;
        T *ub = U + (size_t)slot * NV * P;
        for (int e = a.start[item]; e < a.start[item + 1]; e++) {
            const RefluxRec r = a.recs[e];
            const T dtdx = (T)(dtv / dxp[r.dim]);
            const int t1 = r.dim == 0 ? 1 : 0, t2 = r.dim == 2 ? 1 : 2;
            for (int idx = threadIdx.x; idx < FC * (K1 - K0); idx += NTA) {
                const int k = K0 + idx / FC, tt = idx - (k - K0) * FC;
                const int ta = tt % NB, tb = NDIM == 3 ? tt / NB : 0;
                T f[4];
                const int nf = NDIM == 3 ? 4 : 2;
#pragma unroll
                for (int o = 0; o < 4; o++) {
                    if (o >= nf)
                        break;
                    const int fa = 2 * ta + (o & 1);
                    const int fbb = NDIM == 3 ? 2 * tb + ((o >> 1) & 1) : 0;
                    const int which = (fa / NB) | ((fbb / NB) << 1);
                    const int tl = (fbb % NB) * NB + (fa % NB);
                    f[o] = fb[((size_t)r.fb_fine[which] * NV + k) * FC + (NDIM == 3 ? tl : fa % NB)];
                }
                T mean;
                if constexpr (NDIM == 3)
                    mean = ((f[0] + f[1]) + (f[2] + f[3])) * T(0.25);
                else
                    mean = (f[0] + f[1]) * T(0.5);
                const T fcv = fb[((size_t)r.fb_coarse * NV + k) * FC + tt];
                const T delta = dtdx * (fcv - mean);
                int loc[3] = {0, 0, 0};
                loc[r.dim] = r.side ? NB - 1 : 0;
                loc[t1] = ta;
                if (t2 < NDIM)
                    loc[t2] = tb;
                T *cell = ub + (size_t)k * P + lin<NDIM>(loc[0], loc[1], loc[2]);
                *cell = r.side ? *cell + delta : *cell - delta;
            }
            __syncthreads();  // faces of one block may share edge cells
        }
    }
}

// ---- CFL: per leaf, max over interior cells of max_d |v_d| + c_f,d (FP64)
template <int NDIM, typename T>
__global__ void __launch_bounds__(NTA) k_cfl(CflArgs a)
{
    constexpr int P = FG<NDIM>::P, NI = FG<NDIM>::NI;
    __shared__ double red[NTA / 64];
    const T *U = (const T *)a.U;
    for (int item = blockIdx.x; item < a.nleaves; item += gridDim.x) {
        const int slot = a.leaves[item];
        const T *ub = U + (size_t)slot * NV * P;
        double m = 0.0, cm = 0.0;
        unsigned bad = 0, nonfin = 0;
        for (int i = threadIdx.x; i < NI; i += NTA) {
            const int x = i % NB, y = (i / NB) % NB, z = NDIM == 3 ? i / (NB * NB) : 0;
            const int c = lin<NDIM>(x, y, z);
            double u[NV];
            bool fin = true;
#pragma unroll
            for (int k = 0; k < NV; k++) {
                u[k] = (double)ub[(size_t)k * P + c];
                fin = fin && isfinite(u[k]);
            }
            if (!fin) {
                nonfin++;
                continue;
            }
            double pr;
            bool b;
            const double s = cfl_speed<NDIM>(u, a.gamma, pr, b);
            if (b)
                bad++;
            if (a.cpart) {
                // conduction: kappa T / p = kappa / rho with T = p / rho
                const double r = kappa_of(a.kappa0, a.khalf, pr / u[RHO]) / u[RHO];
                cm = r > cm ? r : cm;
            }
            m = s > m ? s : m;
        }
        if (bad)
            atomicAdd(&a.cnt[2], (unsigned long long)bad);
        if (nonfin)
            atomicAdd(&a.cnt[3], (unsigned long long)nonfin);
        // wave64 shuffle max, then across the 4 waves through LDS
        auto block_max = [&](double v) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                double o = __shfl_xor(v, off, 64);
                v = o > v ? o : v;
            }
            const int w = threadIdx.x >> 6;
            if ((threadIdx.x & 63) == 0)
                red[w] = v;
            __syncthreads();
            double r = red[0];
            for (int i = 1; i < NTA / 64; i++)
                r = red[i] > r ? red[i] : r;
            __syncthreads();
            return r;
        };
        const int pi = a.part_idx ? a.part_idx[item] : item;
        const double mm = block_max(m);
        if (threadIdx.x == 0)
            a.part[pi] = mm;
        if (a.cpart) {
            const double cc = block_max(cm);
            if (threadIdx.x == 0)
                a.cpart[pi] = cc;
        }
    }
}

// ---- time-step record per simulation (one workgroup each)
__global__ void __launch_bounds__(NTA) k_dt(DtArgs a)
{
    __shared__ double red[NTA / 64];
    const int s = blockIdx.x;
    if (s >= a.nsims)
        return;
    const SimRec sr = a.sims[s];
    auto sim_max = [&](const double *part) {
        double m = 0.0;
        // unrolled so that the loads of several iterations are in flight
        // together (the maximum does not depend on the order)
#pragma unroll 8
        for (int i = sr.leaf_lo + (int)threadIdx.x; i < sr.leaf_hi; i += NTA)
            m = part[i] > m ? part[i] : m;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            double o = __shfl_xor(m, off, 64);
            m = o > m ? o : m;
        }
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = m;
        __syncthreads();
        double r = red[0];
        for (int i = 1; i < NTA / 64; i++)
            r = red[i] > r ? red[i] : r;
        __syncthreads();
        return r;
    };
    const double alpha = sim_max(a.part);
    const double kmax = a.cpart ? sim_max(a.cpart) : 0.0;
    if (threadIdx.x == 0) {
        const double dxmin = sr.dxmin;
        double dt = a.cfl * dxmin / (a.ndim * alpha);
        if (a.eta > 0.0) {
            double dr = a.cfl * dxmin * dxmin / (a.ndim * a.eta);
            dt = dr < dt ? dr : dt;
        }
        map_dt r;
        r.dt_sub = 0.0;
        r.nsub = 0;
        r.reserved = 0;
        if (a.cpart && kmax > 0.0) {
            // conduction sub-step limit (Sec. 3.4); the step holds at most
            // cond_max_sub sub-steps
            const double dtc = a.cfl * dxmin * dxmin / (a.ndim * kmax);
            const double cap = a.cond_max_sub * dtc;
            dt = cap < dt ? cap : dt;
            const double ns = ceil(dt / dtc);
            const int nsub = ns < 1.0 ? 1 : (ns > a.cond_max_sub ? a.cond_max_sub : (int)ns);
            r.nsub = nsub;
            r.dt_sub = dt / nsub;
        }
        r.dt = dt;
        r.alpha = alpha;
        if (a.glm_mode == MAP_GLM_PAPER) {
            r.ch = a.cfl * dxmin / dt;
            r.damp = a.cd;
        } else {
            r.ch = alpha;
            r.damp = exp(-dt * r.ch / a.cr);
        }
        a.dt_int[s] = r;
        if (a.dt_out)
            a.dt_out[s] = r;
    }
}

// ---- FP64 totals: per leaf (fixed order), then per simulation (fixed order)
template <int NDIM, typename T>
__global__ void __launch_bounds__(NTA) k_totals_leaf(TotalsArgs a)
{
    constexpr int P = FG<NDIM>::P, NI = FG<NDIM>::NI;
    __shared__ double red[NV][NTA];
    const T *U = (const T *)a.U;
    for (int item = blockIdx.x; item < a.nleaves; item += gridDim.x) {
        const int slot = a.leaves[item];
        const BlockRec br = a.blk[slot];
        const double *dxp = a.lvl_dx + ((size_t)br.sim * (MAXL + 1) + br.level) * 3;
        const double vol = dxp[0] * dxp[1] * (NDIM == 3 ? dxp[2] : 1.0);
        const T *ub = U + (size_t)slot * NV * P;
        double acc[NV];
#pragma unroll
        for (int k = 0; k < NV; k++)
            acc[k] = 0.0;
        for (int i = threadIdx.x; i < NI; i += NTA) {
            const int x = i % NB, y = (i / NB) % NB, z = NDIM == 3 ? i / (NB * NB) : 0;
            const int c = lin<NDIM>(x, y, z);
#pragma unroll
            for (int k = 0; k < NV; k++)
                acc[k] += (double)ub[(size_t)k * P + c] * vol;
        }
#pragma unroll
        for (int k = 0; k < NV; k++)
            red[k][threadIdx.x] = acc[k];
        __syncthreads();
        for (int h = NTA / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h)
#pragma unroll
                for (int k = 0; k < NV; k++)
                    red[k][threadIdx.x] += red[k][threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x < NV)
            a.part[(size_t)item * NV + threadIdx.x] = red[threadIdx.x][0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(NTA) k_totals_sim(TotalsArgs a)
{
    __shared__ double red[NV][NTA];
    const int s = blockIdx.x;
    if (s >= a.nsims)
        return;
    const SimRec sr = a.sims[s];
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; k++)
        acc[k] = 0.0;
    for (int i = sr.leaf_lo + (int)threadIdx.x; i < sr.leaf_hi; i += NTA)
#pragma unroll
        for (int k = 0; k < NV; k++)
            acc[k] += a.part[(size_t)i * NV + k];
#pragma unroll
    for (int k = 0; k < NV; k++)
        red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = NTA / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int k = 0; k < NV; k++)
                red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < NV)
        a.out[(size_t)s * NV + threadIdx.x] = red[threadIdx.x][0];
}

// ---- primitive (rho, v, B, p, psi) -> conserved, e = p/(gamma-1) + rho v^2/2 + B^2/2
template <typename T>
__global__ void __launch_bounds__(NTA) k_prim_to_cons(T *U, size_t nslots, int tile, double gamma)
{
    const size_t total = nslots * (size_t)tile;
    for (size_t i = blockIdx.x * (size_t)NTA + threadIdx.x; i < total; i += (size_t)gridDim.x * NTA) {
        const size_t s = i / tile, c = i - s * tile;
        T *b = U + s * NV * tile + c;
        const double r = b[RHO * (size_t)tile], vx = b[MX * (size_t)tile], vy = b[MY * (size_t)tile],
                     vz = b[MZ * (size_t)tile];
        const double bx = b[BX * (size_t)tile], by = b[BY * (size_t)tile], bz = b[BZ * (size_t)tile];
        const double pr = b[EN * (size_t)tile];
        const double e = pr / (gamma - 1.0) + 0.5 * r * (vx * vx + vy * vy + vz * vz) +
                         0.5 * (bx * bx + by * by + bz * bz);
        b[MX * (size_t)tile] = (T)(r * vx);
        b[MY * (size_t)tile] = (T)(r * vy);
        b[MZ * (size_t)tile] = (T)(r * vz);
        b[EN * (size_t)tile] = (T)e;
    }
}

__global__ void k_clear_u64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0ull;
}

// ------------------------------------------------------------------ launchers
#define DISPATCH(ndim, fp64, KER, ...)                                              \
    do {                                                                            \
        if (ndim == 2) {                                                            \
            if (fp64)                                                               \
                hipLaunchKernelGGL((KER<2, double>), __VA_ARGS__);                  \
            else                                                                    \
                hipLaunchKernelGGL((KER<2, float>), __VA_ARGS__);                   \
        } else {                                                                    \
            if (fp64)                                                               \
                hipLaunchKernelGGL((KER<3, double>), __VA_ARGS__);                  \
            else                                                                    \
                hipLaunchKernelGGL((KER<3, float>), __VA_ARGS__);                   \
        }                                                                           \
    } while (0)

// as DISPATCH, for kernels with an energy-only variant chosen by a.eonly
#define DISPATCH_CFL(ndim, fp64, ...)                                               \
    do {                                                                            \
        if (ndim == 2) {                                                            \
            if (fp64)                                                               \
                hipLaunchKernelGGL((k_restrict<2, double, false, true>), __VA_ARGS__); \
            else                                                                    \
                hipLaunchKernelGGL((k_restrict<2, float, false, true>), __VA_ARGS__); \
        } else {                                                                    \
            if (fp64)                                                               \
                hipLaunchKernelGGL((k_restrict<3, double, false, true>), __VA_ARGS__); \
            else                                                                    \
                hipLaunchKernelGGL((k_restrict<3, float, false, true>), __VA_ARGS__); \
        }                                                                           \
    } while (0)

#define DISPATCH_EO(ndim, fp64, eo, KER, ...)                                       \
    do {                                                                            \
        if (eo) {                                                                   \
            if (ndim == 2) {                                                        \
                if (fp64)                                                           \
                    hipLaunchKernelGGL((KER<2, double, true>), __VA_ARGS__);        \
                else                                                                \
                    hipLaunchKernelGGL((KER<2, float, true>), __VA_ARGS__);         \
            } else {                                                                \
                if (fp64)                                                           \
                    hipLaunchKernelGGL((KER<3, double, true>), __VA_ARGS__);        \
                else                                                                \
                    hipLaunchKernelGGL((KER<3, float, true>), __VA_ARGS__);         \
            }                                                                       \
        } else {                                                                    \
            if (ndim == 2) {                                                        \
                if (fp64)                                                           \
                    hipLaunchKernelGGL((KER<2, double, false>), __VA_ARGS__);       \
                else                                                                \
                    hipLaunchKernelGGL((KER<2, float, false>), __VA_ARGS__);        \
            } else {                                                                \
                if (fp64)                                                           \
                    hipLaunchKernelGGL((KER<3, double, false>), __VA_ARGS__);       \
                else                                                                \
                    hipLaunchKernelGGL((KER<3, float, false>), __VA_ARGS__);        \
            }                                                                       \
        }                                                                           \
    } while (0)

int fill_blocks_per_group(int ndim) { return ndim == 3 ? FG<3>::BPW : FG<2>::BPW; }

hipError_t launch_fill_copy(int ndim, bool fp64, const FillArgs &a, int grid, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    int g = grid > 0 ? (grid < a.nitems ? grid : a.nitems) : a.nitems;
    if (a.eonly && g > SUB_GRID)
        g = SUB_GRID;
    DISPATCH_EO(ndim, fp64, a.eonly, k_fill_copy, dim3(g), dim3(NTA), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_prolong_ghosts(int ndim, bool fp64, const FillArgs &a, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    const int g = a.eonly && a.nitems > SUB_GRID ? SUB_GRID : a.nitems;
    DISPATCH_EO(ndim, fp64, a.eonly, k_prolong_ghosts, dim3(g), dim3(NTA), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_prolong_blocks(int ndim, bool fp64, const FillArgs &a, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    DISPATCH(ndim, fp64, k_prolong_blocks, dim3(a.nitems), dim3(NTA), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_restrict(int ndim, bool fp64, const RestrictArgs &a, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    if (a.cfl) {
        if (a.eonly)
            return hipErrorInvalidValue;
        DISPATCH_CFL(ndim, fp64, dim3(a.nitems), dim3(NTA), 0, s, a);
    } else {
        const int g = a.eonly && a.nitems > SUB_GRID ? SUB_GRID : a.nitems;
        DISPATCH_EO(ndim, fp64, a.eonly, k_restrict, dim3(g), dim3(NTA), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_reflux(int ndim, bool fp64, const RefluxArgs &a, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    const int g = a.eonly && a.nitems > SUB_GRID ? SUB_GRID : a.nitems;
    DISPATCH_EO(ndim, fp64, a.eonly, k_reflux, dim3(g), dim3(NTA), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cfl(int ndim, bool fp64, const CflArgs &a, hipStream_t s)
{
    if (a.nleaves <= 0)
        return hipSuccess;
    DISPATCH(ndim, fp64, k_cfl, dim3(a.nleaves), dim3(NTA), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dt(const DtArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_dt, dim3(a.nsims), dim3(NTA), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_totals(int ndim, bool fp64, const TotalsArgs &a, hipStream_t s)
{
    if (a.nleaves > 0)
        DISPATCH(ndim, fp64, k_totals_leaf, dim3(a.nleaves), dim3(NTA), 0, s, a);
    hipLaunchKernelGGL(k_totals_sim, dim3(a.nsims), dim3(NTA), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_prim_to_cons(bool fp64, void *U, size_t nslots, int tile, double gamma,
                               hipStream_t s)
{
    size_t total = nslots * (size_t)tile;
    int g = (int)((total + NTA - 1) / NTA);
    if (g > 65536)
        g = 65536;
    if (g < 1)
        g = 1;
    if (fp64)
        hipLaunchKernelGGL(k_prim_to_cons<double>, dim3(g), dim3(NTA), 0, s, (double *)U, nslots,
                           tile, gamma);
    else
        hipLaunchKernelGGL(k_prim_to_cons<float>, dim3(g), dim3(NTA), 0, s, (float *)U, nslots, tile,
                           gamma);
    return hipGetLastError();
}

hipError_t launch_clear_u64(unsigned long long *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_u64, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace mapk
