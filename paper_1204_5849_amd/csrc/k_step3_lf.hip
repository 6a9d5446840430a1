// k_step3_lf.hip -- the FP32 TVD-LF instances of the 3-D block update (one
// per limiter and face flux), compiled apart from the WENO stages and the
// FP64 instances so that they can take the instruction scheduler that suits
// them (see the build script).
#include "k_step3.hpp"

namespace mapk {

template <typename T, bool MIXED, bool RESIST, int RS>
static hipError_t launch3_lf(const StepArgs &a, int grid, hipStream_t s)
{
    if (a.limiter == MAP_MINMOD)
        return launch3<T, MIXED, RESIST, SCH_LF, MAP_MINMOD, RS>(a, grid, s);
    if (a.limiter == MAP_VANLEER)
        return launch3<T, MIXED, RESIST, SCH_LF, MAP_VANLEER, RS>(a, grid, s);
    return launch3<T, MIXED, RESIST, SCH_LF, MAP_PAPER_PHI, RS>(a, grid, s);
}

template <typename T, bool MIXED, bool RESIST>
static hipError_t launch3_lf_rs(const StepArgs &a, int grid, hipStream_t s)
{
    if (a.riemann == MAP_HLLC)
        return launch3_lf<T, MIXED, RESIST, MAP_HLLC>(a, grid, s);
    return launch3_lf<T, MIXED, RESIST, MAP_RUSANOV>(a, grid, s);
}

hipError_t launch_step3_lf32(bool resist, const StepArgs &a, int grid, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    return resist ? launch3_lf_rs<float, true, true>(a, grid, s)
                  : launch3_lf_rs<float, true, false>(a, grid, s);
}

}  // namespace mapk
