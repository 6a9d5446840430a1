// cfl.hpp -- the CFL speed of one cell in FP64, shared by the CFL pass, the
// restriction that forms the next cycle's CFL maxima and the 2-D update that
// forms them for the leaves it finalises, so that all three give the same
// value bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include "map_internal.hpp"

namespace mapk {

// the CFL speed of one cell (Sec. 3.7): max over d of |v_d| + c_f,d, in FP64
// from its conserved variables; pr takes the gas pressure and bad is set
// when rho <= 0 or p <= 0
template <int NDIM>
__device__ __forceinline__ double cfl_speed(const double (&u)[NV], double gamma, double &pr,
                                            bool &bad)
{
    // the same arithmetic in every translation unit that includes this
#pragma clang fp contract(off)
    // primitives once per cell, then |v_d| + c_f,d for each d
    const double ir = 1.0 / u[RHO];
    const double vx = u[MX] * ir, vy = u[MY] * ir, vz = u[MZ] * ir;
    const double ke = 0.5 * (u[MX] * vx + u[MY] * vy + u[MZ] * vz);
    const double bb = u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ];
    pr = (gamma - 1.0) * (u[EN] - ke - 0.5 * bb);
    bad = !(u[RHO] > 0.0) || !(pr > 0.0);
    const double a2 = gamma * pr * ir, sab = a2 + bb * ir;
    auto fast = [&](double vd, double Bd) {
        double disc = sab * sab - 4.0 * a2 * (Bd * Bd) * ir;
        disc = disc < 0.0 ? 0.0 : disc;
        double cf2 = 0.5 * (sab + sqrt(disc));
        cf2 = cf2 < 0.0 ? 0.0 : cf2;
        return fabs(vd) + sqrt(cf2);
    };
    double s = fast(vx, u[BX]);
    const double s1 = fast(vy, u[BY]);
    s = s1 > s ? s1 : s;
    if constexpr (NDIM == 3) {
        const double s2 = fast(vz, u[BZ]);
        s = s2 > s ? s2 : s;
    }
    return s;
}

}  // namespace mapk
