// kernels.hpp -- kernel argument records and launch entry points (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "map_internal.hpp"

namespace mapk {

// what one launch of a block-update kernel computes: the TVD-LF step
// (Sec. 3.2), or one stage of WENO with TVD Runge-Kutta 2 (Sec. 3.3):
// stage 1 u1 = u + dt L(u); stage 2 (u + u1 + dt L(u1)) / 2 with the psi
// damping of the whole step
enum { SCH_LF = 0, SCH_WENO1 = 1, SCH_WENO2 = 2 };

struct StepArgs {
    const void *Uin;
    void *Uout;
    const void *Ubase;      // WENO stage 2: u^n, read at the updated cells only (may be Uout)
    const int32_t *leaves;  // leaf slots processed by this launch
    int nleaves;
    int nitems;             // work items (groups of blocks per workgroup)
    const BlockRec *blk;
    const map_dt *dt;
    const double *lvl_dx;
    const int32_t *fbidx;
    const Desc *desc;       // ghost descriptors: neighbour cells are read from Uin in place
    void *fbuf;
    unsigned long long *cnt;
    double gamma, eta;
    int eglm, limiter, riemann;
    // workgroup shape of the update: 2-D LF / WENO, 0 = 14 blocks in 4 waves,
    // 1 = 7 blocks in 2 waves; 3-D FP32 LF / WENO, 0 = compiled for two
    // workgroups per CU (256 registers per lane), 1 = for one (512)
    int shape;
    // 2-D LF: with cfl_on, the next cycle's CFL maximum of each leaf whose
    // cfl_leaf[slot] >= 0 (a leaf without parent that no reflux changes) is
    // formed from the values the update writes, into cfl_part[cfl_leaf[slot]]
    int cfl_on;
    const int32_t *cfl_leaf;
    double *cfl_part;
};

// energy-only passes of a conduction sub-step (eonly = 1): only the energy
// moves, and blocks of simulations with sub >= dt[sim].nsub are skipped
struct FillArgs {
    void *U;
    const Desc *desc;
    const BlockRec *blk;
    const int32_t *parent;
    const int32_t *list;       // prolongation: slots of the launch
    const uint32_t *list_mask; // prolongation: prolongated ghost directions per list entry
    const int32_t *copy_list;  // copies: slots (null: slot = index)
    const FrameSel *copy_sel;  // copies: ghost cells to fill per list entry (null: all)
    int slot_base, slot_end, nitems;  // copies: index range [slot_base, slot_end)
    const map_dt *dt;
    int eonly, sub, nsims;
};

struct RestrictArgs {
    void *U;
    const int32_t *list;
    const int32_t *children;
    int nitems;
    const BlockRec *blk;
    const map_dt *dt;
    int eonly, sub, nsims;
    // with cfl set: the CFL maxima of the leaf children, from the values
    // the restriction reads, into part (by leaf index, from leaf_of), and
    // the cells with rho <= 0 or p <= 0, or not finite, into cnt[2], cnt[3]
    int cfl;
    int per_child;  // items are parents x 2^d, one child each (else one parent each)
    double *part;
    const int32_t *leaf_of;
    unsigned long long *cnt;
    double gamma;
};

struct RefluxArgs {
    void *U;
    const int32_t *slots;
    const int32_t *start;
    const RefluxRec *recs;
    const BlockRec *blk;
    const map_dt *dt;
    const double *lvl_dx;
    const void *fbuf;
    int nitems;
    int eonly, sub, nsims;  // conduction sub-step: energy only, dt_sub
};

struct CflArgs {
    const void *U;
    const int32_t *leaves;
    int nleaves;
    double *part;
    const int32_t *part_idx;  // part index of each listed leaf (null: its list index)
    double *cpart;  // conduction: per leaf max kappa T / p (null: off)
    unsigned long long *cnt;
    double gamma, kappa0;
    int khalf;      // 2 x kappa exponent
};

struct DtArgs {
    const double *part;
    const double *cpart;  // null: no conduction
    const SimRec *sims;
    map_dt *dt_int;
    map_dt *dt_out;  // optional copy
    int nsims, ndim, glm_mode, cond_max_sub;
    double cfl, cd, cr, eta;
};

// one conduction sub-step (Sec. 3.4)
struct CondArgs {
    void *U;
    void *S;               // scratch state: its energy plane takes the new energy
    const int32_t *list;   // leaves
    int nitems;
    const BlockRec *blk;
    const Desc *desc;
    const map_dt *dt;
    const double *lvl_dx;
    const int32_t *fbidx;
    void *fbuf;
    double gamma, kappa0;
    int khalf, mode, sub, nsims;
};

// a conduction sub-step beyond the subcycle of every simulation: the
// sub-step's kernels return at once (they are launched whatever nsub is, so
// that the launch sequence does not depend on data)
__device__ __forceinline__ bool sub_idle(const map_dt *dt, int nsims, int sub)
{
    for (int s = 0; s < nsims; s++)
        if (sub < dt[s].nsub)
            return false;
    return true;
}

// grid of a conduction sub-step launch: a persistent grid of at most this
// many workgroups, so that an idle sub-step costs a few thousand tiny
// workgroups rather than one per block
constexpr int SUB_GRID = 2048;

struct TotalsArgs {
    const void *U;
    const int32_t *leaves;
    int nleaves;
    const BlockRec *blk;
    const double *lvl_dx;
    double *part;
    const SimRec *sims;
    double *out;
    int nsims, ndim;
};

struct EstArgs {
    const void *U;
    const Desc *desc;
    const BlockRec *blk;
    double *err;
    int nslots;
    map_estimator est;
};

struct RemapArgs {
    void *Udst;
    const void *Usrc;
    const int32_t *map;   // by destination slot: source slot or -1
    size_t tile_bytes;    // NV x padded cells x word
    int nslots;
};

// launchers (defined in the .hip files); return hipError_t of the launch
hipError_t launch_step2(bool fp64, bool resist, int sch, const StepArgs &a, int grid, hipStream_t s);
hipError_t launch_step3(bool fp64, bool resist, int sch, const StepArgs &a, int grid, hipStream_t s);
hipError_t launch_step3_ilp(int sch, const StepArgs &a, int grid, hipStream_t s);
hipError_t launch_step_mmc(int ndim, bool fp64, const StepArgs &a, double alpha_unused, int grid,
                           hipStream_t s);
hipError_t launch_step_mmc3(bool fp64, bool resist, const StepArgs &a, int grid, hipStream_t s);
// blocks per workgroup of the batched update for a workgroup shape (StepArgs::shape)
int step_blocks_per_group(int ndim, int scheme, int shape);
hipError_t launch_fill_copy(int ndim, bool fp64, const FillArgs &a, int grid, hipStream_t s);
int fill_blocks_per_group(int ndim);
hipError_t launch_prolong_ghosts(int ndim, bool fp64, const FillArgs &a, hipStream_t s);
hipError_t launch_prolong_blocks(int ndim, bool fp64, const FillArgs &a, hipStream_t s);
hipError_t launch_restrict(int ndim, bool fp64, const RestrictArgs &a, hipStream_t s);
hipError_t launch_reflux(int ndim, bool fp64, const RefluxArgs &a, hipStream_t s);
hipError_t launch_cfl(int ndim, bool fp64, const CflArgs &a, hipStream_t s);
hipError_t launch_dt(const DtArgs &a, hipStream_t s);
hipError_t launch_totals(int ndim, bool fp64, const TotalsArgs &a, hipStream_t s);
hipError_t launch_prim_to_cons(bool fp64, void *U, size_t ncell_per_var_total, int tile,
                               double gamma, hipStream_t s);
hipError_t launch_clear_u64(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_estimate(int ndim, bool fp64, const EstArgs &a, hipStream_t s);
hipError_t launch_conduct(int ndim, bool fp64, const CondArgs &a, hipStream_t s);
hipError_t launch_cond_commit(int ndim, bool fp64, const CondArgs &a, hipStream_t s);
hipError_t launch_remap_copy(const RemapArgs &a, hipStream_t s);

}  // namespace mapk
