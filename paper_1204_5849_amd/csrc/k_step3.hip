// k_step3.hip -- launches of the 3-D block update: the FP32 resistive LF
// step and first WENO stage are instantiated in k_step3_ilp.hip, every other
// instance here.
#include "k_step3.hpp"

namespace mapk {

template <typename T, bool MIXED, bool RESIST, int RS>
static hipError_t launch3_weno(int sch, const StepArgs &a, int grid, hipStream_t s)
{
    if (sch == SCH_WENO1)
        return launch3<T, MIXED, RESIST, SCH_WENO1, MAP_MINMOD, RS>(a, grid, s);
    return launch3<T, MIXED, RESIST, SCH_WENO2, MAP_MINMOD, RS>(a, grid, s);
}

template <typename T, bool MIXED, bool RESIST, int RS>
static hipError_t launch3_lf(const StepArgs &a, int grid, hipStream_t s)
{
    if (a.limiter == MAP_MINMOD)
        return launch3<T, MIXED, RESIST, SCH_LF, MAP_MINMOD, RS>(a, grid, s);
    if (a.limiter == MAP_VANLEER)
        return launch3<T, MIXED, RESIST, SCH_LF, MAP_VANLEER, RS>(a, grid, s);
    return launch3<T, MIXED, RESIST, SCH_LF, MAP_PAPER_PHI, RS>(a, grid, s);
}

template <typename T, bool MIXED, bool RESIST, int RS>
static hipError_t launch3_any(int sch, const StepArgs &a, int grid, hipStream_t s)
{
    if (sch == SCH_LF)
        return launch3_lf<T, MIXED, RESIST, RS>(a, grid, s);
    return launch3_weno<T, MIXED, RESIST, RS>(sch, a, grid, s);
}

template <typename T, bool MIXED, bool RESIST>
static hipError_t launch3_rs(int sch, const StepArgs &a, int grid, hipStream_t s)
{
    if constexpr (MIXED && RESIST) {
        // FP32 resistive: only the second WENO stage is instantiated here
        // (each instance lives in one translation unit, so the scheduler it
        // was compiled with is the one that runs)
        if (a.riemann == MAP_HLLC)
            return launch3<T, MIXED, RESIST, SCH_WENO2, MAP_MINMOD, MAP_HLLC>(a, grid, s);
        return launch3<T, MIXED, RESIST, SCH_WENO2, MAP_MINMOD, MAP_RUSANOV>(a, grid, s);
    } else {
        if (a.riemann == MAP_HLLC)
            return launch3_any<T, MIXED, RESIST, MAP_HLLC>(sch, a, grid, s);
        return launch3_any<T, MIXED, RESIST, MAP_RUSANOV>(sch, a, grid, s);
    }
}

hipError_t launch_step3(bool fp64, bool resist, int sch, const StepArgs &a, int grid, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    if (!fp64 && resist && sch != SCH_WENO2)
        return launch_step3_ilp(sch, a, grid, s);
    if (fp64)
        return resist ? launch3_rs<double, false, true>(sch, a, grid, s)
                      : launch3_rs<double, false, false>(sch, a, grid, s);
    return resist ? launch3_rs<float, true, true>(sch, a, grid, s)
                  : launch3_rs<float, true, false>(sch, a, grid, s);
}

}  // namespace mapk
