// physics.hpp -- device-side pointwise EGLM-MHD physics: pressure, fluxes,
// fast speeds and limiters (paper Sec. 2 and Sec. 3).  T = double for the
// FP64 path; T = float with MIXED = true for the FP32 path, where the
// pressure is recovered in FP64 from the FP32 conserved variables (the
// products of FP32 numbers are exact in FP64, so the cancellation in
// e - rho v^2/2 - B^2/2 at low plasma beta costs no precision).
#pragma once

#include <hip/hip_runtime.h>

#include "map_internal.hpp"

namespace mapk {

template <typename T>
struct Num;

template <>
struct Num<double> {
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
};

template <>
struct Num<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
};

// conduction coefficient kappa = kappa0 T^(khalf/2) (Sec. 3.4): whole
// powers by repeated multiplication, then one square root for a half power
__device__ __forceinline__ double kappa_of(double kappa0, int khalf, double T)
{
    double q = 1.0;
    for (int i = 0; i < khalf / 2; i++)
        q = q * T;
    if (khalf & 1)
        q = q * sqrt(T);
    return kappa0 * q;
}

template <typename T>
__device__ __forceinline__ T sgn_of(T a)
{
    return a > T(0) ? T(1) : (a < T(0) ? T(-1) : T(0));
}

// minmod(a,b) = sgn(a) max(0, min(|a|, sgn(a) b))  (eq. minmod)
template <typename T>
__device__ __forceinline__ T lim_minmod(T a, T b)
{
    T s = sgn_of(a);
    T m = fabs(a);
    T t = s * b;
    m = t < m ? t : m;
    m = m < T(0) ? T(0) : m;
    return s * m;
}

// in FP32 the same value is the median of (a, b, 0): the smaller magnitude
// when a and b share a sign, zero otherwise -- one v_med3_f32 instruction
template <>
__device__ __forceinline__ float lim_minmod<float>(float a, float b)
{
    return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}

// slope / flux limiter, chosen at compile time (kernels are instantiated
// per limiter so that no per-call dispatch sits in the cell loop): minmod,
// van Leer (ab + |ab|)/(a + b), or the literal flux limiter of Sec. 3.1 in
// ratio-free form phi(a/b) b
template <int KIND, typename T>
__device__ __forceinline__ T limiter(T a, T b)
{
    if constexpr (KIND == MAP_MINMOD) {
        return lim_minmod(a, b);
    } else if constexpr (KIND == MAP_VANLEER) {
        T ab = a * b;
        return ab <= T(0) ? T(0) : Num<T>::div(ab + fabs(ab), a + b);
    } else {
        return fabs(a) <= fabs(b) ? a : b;
    }
}

template <typename T, bool MIXED>
struct Phys {
    T gamma, gm1;
    double gm1d;

    // p = (gamma - 1)(e - rho v^2/2 - B^2/2); ir = 1/rho, v = m ir.
    // MIXED: recovered in FP64 from the FP32 conserved variables, whose
    // products are exact in FP64, so the cancellation at low beta costs no
    // precision.
    __device__ __forceinline__ T pressure(const T u[NV], T ir, T vx, T vy, T vz, T me) const
    {
        if constexpr (MIXED) {
            double r = (double)ir;
            r = r * (2.0 - (double)u[RHO] * r);  // one Newton step on 1/rho
            double m2 = (double)u[MX] * (double)u[MX] + (double)u[MY] * (double)u[MY] +
                        (double)u[MZ] * (double)u[MZ];
            double b2 = (double)u[BX] * (double)u[BX] + (double)u[BY] * (double)u[BY] +
                        (double)u[BZ] * (double)u[BZ];
            return (T)(gm1d * (((double)u[EN] - 0.5 * m2 * r) - 0.5 * b2));
        } else {
            T ke = T(0.5) * (u[MX] * vx + u[MY] * vy + u[MZ] * vz);
            return gm1 * (u[EN] - ke - me);
        }
    }

    __device__ __forceinline__ bool admissible(const T u[NV]) const
    {
        if (!(u[RHO] > T(0)))
            return false;
        T ir = Num<T>::rcp(u[RHO]);
        T vx = u[MX] * ir, vy = u[MY] * ir, vz = u[MZ] * ir;
        T me = T(0.5) * (u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ]);
        return pressure(u, ir, vx, vy, vz, me) > T(0);
    }

    // EGLM flux along D (MHD-1..MHD-5); returns |v_D| + c_f,D if SPEED
    template <int D, bool SPEED>
    __device__ __forceinline__ T flux(const T u[NV], T ch2, T f[NV]) const
    {
        T ir = Num<T>::rcp(u[RHO]);
        T v[3] = {u[MX] * ir, u[MY] * ir, u[MZ] * ir};
        const T B[3] = {u[BX], u[BY], u[BZ]};
        T bb = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
        T me = T(0.5) * bb;
        T pr = pressure(u, ir, v[0], v[1], v[2], me);
        T pt = pr + me;
        T vd = v[D], Bd = B[D];
        T vb = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
        f[RHO] = u[MX + D];
#pragma unroll
        for (int j = 0; j < 3; j++)
            f[MX + j] = u[MX + j] * vd - B[j] * Bd;
        f[MX + D] = f[MX + D] + pt;
#pragma unroll
        for (int j = 0; j < 3; j++)
            f[BX + j] = B[j] * vd - Bd * v[j];
        f[BX + D] = u[PSI];
        f[EN] = (u[EN] + pt) * vd - Bd * vb;
        f[PSI] = ch2 * Bd;
        if constexpr (SPEED) {
            T a2 = gamma * pr * ir;
            T b2 = bb * ir;
            T s = a2 + b2;
            T disc = s * s - T(4) * a2 * (Bd * Bd) * ir;
            disc = disc < T(0) ? T(0) : disc;
            T cf2 = T(0.5) * (s + Num<T>::sqrt_(disc));
            cf2 = cf2 < T(0) ? T(0) : cf2;
            return fabs(vd) + Num<T>::sqrt_(cf2);
        } else {
            return T(0);
        }
    }
};

// primitive quantities of one state, computed once and shared by the
// admissibility test, the flux and the fast speed of that state
template <typename T>
struct Prim {
    T ir, vx, vy, vz, bb, p;
};

template <typename T, bool MIXED>
__device__ __forceinline__ void prim_of(const Phys<T, MIXED> &ph, const T u[NV], Prim<T> &w)
{
    w.ir = Num<T>::rcp(u[RHO]);
    w.vx = u[MX] * w.ir;
    w.vy = u[MY] * w.ir;
    w.vz = u[MZ] * w.ir;
    w.bb = u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ];
    w.p = ph.pressure(u, w.ir, w.vx, w.vy, w.vz, T(0.5) * w.bb);
}

template <typename T>
__device__ __forceinline__ bool admissible_w(const T u[NV], const Prim<T> &w)
{
    return u[RHO] > T(0) && w.p > T(0);
}

// EGLM flux along dimension d from a state and its primitives.  d may differ
// between lanes (a wave that serves faces of several orientations); with a
// constant d the selects fold away, so every caller forms the same
// arithmetic and a flux does not depend on which lane evaluated it.
template <typename T>
__device__ __forceinline__ void flux_sel(const T u[NV], const Prim<T> &w, int d, T ch2, T f[NV])
{
    const T me = T(0.5) * w.bb;
    const T pt = w.p + me;
    const T vd = d == 0 ? w.vx : (d == 1 ? w.vy : w.vz);
    const T Bd = d == 0 ? u[BX] : (d == 1 ? u[BY] : u[BZ]);
    const T vb = w.vx * u[BX] + w.vy * u[BY] + w.vz * u[BZ];
    f[RHO] = d == 0 ? u[MX] : (d == 1 ? u[MY] : u[MZ]);
    f[MX] = u[MX] * vd - u[BX] * Bd;
    f[MY] = u[MY] * vd - u[BY] * Bd;
    f[MZ] = u[MZ] * vd - u[BZ] * Bd;
    f[MX] = d == 0 ? f[MX] + pt : f[MX];
    f[MY] = d == 1 ? f[MY] + pt : f[MY];
    f[MZ] = d == 2 ? f[MZ] + pt : f[MZ];
    f[BX] = d == 0 ? u[PSI] : u[BX] * vd - Bd * w.vx;
    f[BY] = d == 1 ? u[PSI] : u[BY] * vd - Bd * w.vy;
    f[BZ] = d == 2 ? u[PSI] : u[BZ] * vd - Bd * w.vz;
    f[EN] = (u[EN] + pt) * vd - Bd * vb;
    f[PSI] = ch2 * Bd;
}

template <int D, typename T>
__device__ __forceinline__ void flux_w(const T u[NV], const Prim<T> &w, T ch2, T f[NV])
{
    flux_sel(u, w, D, ch2, f);
}

// fast magnetosonic speed c_f,d from a state and its primitives
template <typename T>
__device__ __forceinline__ T fast_sel(const T u[NV], const Prim<T> &w, int d, T gamma)
{
    const T a2 = gamma * w.p * w.ir;
    const T b2 = w.bb * w.ir;
    const T s = a2 + b2;
    const T Bd = d == 0 ? u[BX] : (d == 1 ? u[BY] : u[BZ]);
    T disc = s * s - T(4) * a2 * (Bd * Bd) * w.ir;
    disc = disc < T(0) ? T(0) : disc;
    T cf2 = T(0.5) * (s + Num<T>::sqrt_(disc));
    cf2 = cf2 < T(0) ? T(0) : cf2;
    return Num<T>::sqrt_(cf2);
}

// |v_d| + c_f,d from a state and its primitives (d as in flux_sel)
template <typename T>
__device__ __forceinline__ T speed_sel(const T u[NV], const Prim<T> &w, int d, T gamma)
{
    const T vd = d == 0 ? w.vx : (d == 1 ? w.vy : w.vz);
    return fabs(vd) + fast_sel(u, w, d, gamma);
}

template <int D, typename T>
__device__ __forceinline__ T speed_w(const T u[NV], const Prim<T> &w, T gamma)
{
    return speed_sel(u, w, D, gamma);
}

}  // namespace mapk
