// k_step3_ilp.hip -- the FP32 resistive instances of the 3-D block update
// that run faster under LLVM's ILP-first instruction scheduler: the TVD-LF
// step (one per limiter and face flux) and the first WENO stage.  The
// others stay in k_step3.hip with the default scheduler (see the build
// script).
#include "k_step3.hpp"

namespace mapk {

template <int RS>
static hipError_t launch3_ilp(int sch, const StepArgs &a, int grid, hipStream_t s)
{
    if (sch == SCH_WENO1)
        return launch3<float, true, true, SCH_WENO1, MAP_MINMOD, RS>(a, grid, s);
    if (a.limiter == MAP_MINMOD)
        return launch3<float, true, true, SCH_LF, MAP_MINMOD, RS>(a, grid, s);
    if (a.limiter == MAP_VANLEER)
        return launch3<float, true, true, SCH_LF, MAP_VANLEER, RS>(a, grid, s);
    return launch3<float, true, true, SCH_LF, MAP_PAPER_PHI, RS>(a, grid, s);
}

// FP32, resistive, LF or the first WENO stage
hipError_t launch_step3_ilp(int sch, const StepArgs &a, int grid, hipStream_t s)
{
    if (a.nitems <= 0)
        return hipSuccess;
    if (a.riemann == MAP_HLLC)
        return launch3_ilp<MAP_HLLC>(sch, a, grid, s);
    return launch3_ilp<MAP_RUSANOV>(sch, a, grid, s);
}

}  // namespace mapk
