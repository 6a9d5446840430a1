// k_regrid.hip -- device side of a regrid (paper Sec. 4.5): the error
// estimator per block, and the copy of surviving blocks onto a new tree.
#include "kernels.hpp"
#include "tile.hpp"

#pragma clang fp contract(off)

namespace mapk {

namespace {
constexpr int NTE = 256;
// the estimator's workgroup: in 3-D 512 threads per block (8 waves), so that
// the two blocks whose 64 KB FP64 staging tiles fit in a CU's LDS keep four
// waves per SIMD over their long FP64 chains (3.91 -> 2.68 ms on the Harris
// sheet against 256 threads); in 2-D (400 cells) 256
constexpr int nt_est(int ndim) { return ndim == 3 ? 512 : 256; }
}

// value of criterion i at a padded cell of block `slot` (read where the
// ghost descriptors point), in FP64
template <int NDIM, typename T>
__device__ __forceinline__ double est_value(const EstArgs &a, int i, int slot, int x, int y, int z)
{
    constexpr int P = tile_cells<NDIM>();
    const T *p = (const T *)a.U + cell_src<NDIM>(a.desc, slot, x, y, z);
    if (a.est.mode[i] == MAP_EST_BMAG) {
        const double bx = (double)p[BX * P], by = (double)p[BY * P], bz = (double)p[BZ * P];
        return sqrt(bx * bx + by * by + bz * bz);
    }
    return (double)p[(size_t)a.est.var[i] * P];
}

// largest estimate over the interior and the first ghost ring of each block,
// maximum over the criteria; one workgroup per block.  Each criterion's value
// is formed once per padded cell (ghosts read where the descriptors point)
// and staged in LDS; the stencil then runs on LDS.
template <int NDIM, typename T>
__global__ void __launch_bounds__(nt_est(NDIM)) k_estimate(EstArgs a)
{
    constexpr int NTEST = nt_est(NDIM);
    constexpr int PT = tile_cells<NDIM>();
    __shared__ double sv[PT];
    __shared__ double red[NTEST / 64];
    constexpr int E = NB + 2;
    constexpr int NE = NDIM == 3 ? E * E * E : E * E;
    const int st[3] = {1, PD, PD * PD};
    for (int slot = blockIdx.x; slot < a.nslots; slot += gridDim.x) {
        const int level = a.blk[slot].level;
        const double scale = pow(a.est.ratio, a.est.xi * (level - 1));
        double best = 0.0;
        for (int i = 0; i < a.est.ncrit; i++) {
            for (int c = threadIdx.x; c < PT; c += NTEST) {
                const int x = c % PD - NG, y = (c / PD) % PD - NG;
                const int z = NDIM == 3 ? c / (PD * PD) - NG : 0;
                sv[c] = est_value<NDIM, T>(a, i, slot, x, y, z);
            }
            __syncthreads();
            for (int e = threadIdx.x; e < NE; e += NTEST) {
                const int x = e % E - 1, y = (e / E) % E - 1, z = NDIM == 3 ? e / (E * E) - 1 : 0;
                const int c = lin<NDIM>(x, y, z);
                const double v = sv[c];
                double s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int d = 0; d < NDIM; d++) {
                    const double vp = sv[c + st[d]], vm = sv[c - st[d]];
                    s1 += (vp - vm) * (vp - vm);
                    s2 += (vp - 2.0 * v + vm) * (vp - 2.0 * v + vm);
                }
                const double d1 = 0.5 * sqrt(3.0) * sqrt(s1);
                const double d2 = sqrt(s2);
                const double av = fabs(v) + a.est.eps[i];
                const double est =
                    (a.est.bias * d1 / av + (1.0 - a.est.bias) * d2 / (d1 + a.est.filt * av)) * scale;
                best = est > best ? est : best;
            }
            __syncthreads();  // sv is restaged for the next criterion / block
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(best, off, 64);
            best = o > best ? o : best;
        }
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            double r = red[0];
            for (int w = 1; w < NTEST / 64; w++)
                r = red[w] > r ? red[w] : r;
            a.err[slot] = r;
        }
        __syncthreads();
    }
}

// padded tiles of the blocks present in both trees, 16 bytes per thread
__global__ void __launch_bounds__(NTE) k_remap_copy(RemapArgs a)
{
    const size_t n16 = a.tile_bytes / 16;
    for (int slot = blockIdx.x; slot < a.nslots; slot += gridDim.x) {
        const int src = a.map[slot];
        if (src < 0)
            continue;
        const uint4 *s = (const uint4 *)((const char *)a.Usrc + (size_t)src * a.tile_bytes);
        uint4 *d = (uint4 *)((char *)a.Udst + (size_t)slot * a.tile_bytes);
        for (size_t i = threadIdx.x; i < n16; i += NTE)
            d[i] = s[i];
    }
}

hipError_t launch_estimate(int ndim, bool fp64, const EstArgs &a, hipStream_t s)
{
    if (a.nslots <= 0)
        return hipSuccess;
    if (ndim == 2) {
        if (fp64)
            hipLaunchKernelGGL((k_estimate<2, double>), dim3(a.nslots), dim3(nt_est(2)), 0, s, a);
        else
            hipLaunchKernelGGL((k_estimate<2, float>), dim3(a.nslots), dim3(nt_est(2)), 0, s, a);
    } else {
        if (fp64)
            hipLaunchKernelGGL((k_estimate<3, double>), dim3(a.nslots), dim3(nt_est(3)), 0, s, a);
        else
            hipLaunchKernelGGL((k_estimate<3, float>), dim3(a.nslots), dim3(nt_est(3)), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_remap_copy(const RemapArgs &a, hipStream_t s)
{
    if (a.nslots <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_remap_copy, dim3(a.nslots), dim3(NTE), 0, s, a);
    return hipGetLastError();
}

}  // namespace mapk
