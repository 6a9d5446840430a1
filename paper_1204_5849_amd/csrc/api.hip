// api.hip -- the extern "C" entry points of libmap.so: argument checks, the
// device binding of the planned tables, stage launches (batched persistent or
// one launch per block), the step cycle, its HIP-graph capture and the launch
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "keymap.hpp"
#include "plan.hpp"

using namespace mapk;

namespace {

thread_local std::string g_err;

map_status fail(map_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(MAP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

template <typename X>
X *dptr(map_ctx *c, size_t off)
{
    return reinterpret_cast<X *>(c->wsp + off);
}

map_status need_bound(map_ctx *c)
{
    if (!c)
        return fail(MAP_EINVAL, "null context");
    if (!c->bound)
        return fail(MAP_ESTATE, "workspace not bound (call map_bind_workspace first)");
    return MAP_OK;
}

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---- fixed device scratch of map_totals_static --------------------------
// The per-leaf partial sums of the totals for callers that cannot allocate
// (graph capture, serving loops): one array per GPU, held until the process
// ends, shared by every call on that GPU.  Host code never uses the array's
// name as an address: the device address of each GPU's copy is taken once,
// with that GPU current, by hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) double scratch[MAP_STATIC_SCRATCH_DOUBLES];
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// the current device's scratch address, taken on first use on that device
map_status scratch_of_current_device(double **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(MAP_EINVAL, "device index " + std::to_string(dev) + " out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr)
            return fail(MAP_EHIP, "hipGetSymbolAddress returned a null scratch address");
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return MAP_OK;
}

bool fp64(const map_ctx *c) { return c->p.precision == MAP_FP64; }

// Ghost fill: same-level copies, then prolongation level by level (coarse to
// fine).  `all`: the copies fill every slot's ghost frame; otherwise only
// the frames the prolongation reads (the step reads same-level neighbour
// interiors in place).
map_status run_fill(map_ctx *c, void *U, hipStream_t s, bool all, int eonly_sub = -1,
                    const map_dt *dt = nullptr)
{
    FillArgs a{};
    a.U = U;
    a.dt = dt ? dt : dptr<map_dt>(c, c->ws.dt);  // energy-only passes: the subcycle's records
    a.eonly = eonly_sub >= 0;
    a.sub = eonly_sub;
    a.nsims = (int)c->sims.size();
    a.desc = dptr<Desc>(c, c->ws.desc);
    a.blk = dptr<BlockRec>(c, c->ws.blocks);
    a.parent = dptr<int32_t>(c, c->ws.parent);
    a.copy_list = all ? nullptr : dptr<int32_t>(c, c->ws.frame_list);
    a.copy_sel = all ? nullptr : dptr<FrameSel>(c, c->ws.frame_sel);
    const int ncopy = all ? c->nslots : (int)c->frame_list.size();
    const int bpw = fill_blocks_per_group(c->nd);
    if (c->launch_mode == MAP_LAUNCH_PER_BLOCK) {
        for (int i = 0; i < ncopy; i++) {
            a.slot_base = i;
            a.slot_end = i + 1;
            a.nitems = 1;
            HIPCHK(launch_fill_copy(c->nd, fp64(c), a, 1, s));
        }
    } else if (ncopy > 0) {
        a.slot_base = 0;
        a.slot_end = ncopy;
        a.nitems = (ncopy + bpw - 1) / bpw;
        HIPCHK(launch_fill_copy(c->nd, fp64(c), a, c->grid_fill, s));
    }
    for (int l = 2; l <= c->lmax; l++) {
        int lo = c->prolong_off[l], hi = c->prolong_off[l + 1];
        if (hi <= lo)
            continue;
        a.list = dptr<int32_t>(c, c->ws.prolong_list) + lo;
        a.list_mask = dptr<uint32_t>(c, c->ws.prolong_mask) + lo;
        a.nitems = hi - lo;
        HIPCHK(launch_prolong_ghosts(c->nd, fp64(c), a, s));
    }
    return MAP_OK;
}

// restriction of every parent, finest level first; with cfl, the leaf
// children's CFL maxima into the per-leaf parts as well
map_status run_restrict(map_ctx *c, void *U, hipStream_t s, int eonly_sub = -1, bool cfl = false,
                        const map_dt *dt = nullptr)
{
    RestrictArgs a{};
    a.U = U;
    a.children = dptr<int32_t>(c, c->ws.children);
    a.blk = dptr<BlockRec>(c, c->ws.blocks);
    a.dt = dt ? dt : dptr<map_dt>(c, c->ws.dt);  // energy-only passes: the subcycle's records
    a.eonly = eonly_sub >= 0;
    a.sub = eonly_sub;
    a.nsims = (int)c->sims.size();
    a.cfl = cfl;
    a.part = dptr<double>(c, c->ws.cfl_part);
    a.leaf_of = dptr<int32_t>(c, c->ws.leaf_of);
    a.cnt = dptr<unsigned long long>(c, c->ws.counters);
    a.gamma = c->p.gamma;
    for (int l = c->lmax - 1; l >= 1; l--) {
        int lo = c->restrict_off[l], hi = c->restrict_off[l + 1];
        if (hi <= lo)
            continue;
        a.list = dptr<int32_t>(c, c->ws.restrict_list) + lo;
        // a level with fewer parents than CUs (or the tuned split) takes one
        // workgroup per child
        a.per_child = hi - lo < (c->restrict_split >= 0 ? c->restrict_split : c->ncu);
        a.nitems = (hi - lo) * (a.per_child ? (c->nd == 3 ? 8 : 4) : 1);
        HIPCHK(launch_restrict(c->nd, fp64(c), a, s));
    }
    return MAP_OK;
}

// the dt records of every simulation from the per-leaf parts into dt_int
// (the first record buffer if null) and, if given, dt_out
map_status run_dt(map_ctx *c, map_dt *dt_out, hipStream_t s, map_dt *dt_int = nullptr)
{
    const bool cond = c->p.cond_mode != MAP_COND_OFF;
    DtArgs d{};
    d.part = dptr<double>(c, c->ws.cfl_part);
    d.cpart = cond ? dptr<double>(c, c->ws.cond_part) : nullptr;
    d.cond_max_sub = c->p.cond_max_sub;
    d.sims = dptr<SimRec>(c, c->ws.sims);
    d.dt_int = dt_int ? dt_int : dptr<map_dt>(c, c->ws.dt);
    d.dt_out = dt_out;
    d.nsims = (int)c->sims.size();
    d.ndim = c->nd;
    d.glm_mode = c->p.glm_mode;
    d.cfl = c->p.cfl;
    d.cd = c->p.glm_cd;
    d.cr = c->p.glm_cr;
    d.eta = c->p.eta;
    HIPCHK(launch_dt(d, s));
    return MAP_OK;
}

// the per-leaf CFL parts of every leaf of U, then the dt records
map_status run_cfl(map_ctx *c, const void *U, map_dt *dt_out, hipStream_t s,
                   map_dt *dt_int = nullptr)
{
    CflArgs a{};
    a.U = U;
    a.cnt = dptr<unsigned long long>(c, c->ws.counters);
    a.gamma = c->p.gamma;
    const bool cond = c->p.cond_mode != MAP_COND_OFF;
    a.kappa0 = c->p.kappa0;
    a.khalf = (int)(2.0 * c->p.kappa_exp + 0.5);
    if (c->launch_mode == MAP_LAUNCH_PER_BLOCK) {
        for (int i = 0; i < c->nleaves; i++) {
            a.leaves = dptr<int32_t>(c, c->ws.leaves) + i;
            a.nleaves = 1;
            a.part = dptr<double>(c, c->ws.cfl_part) + i;
            a.cpart = cond ? dptr<double>(c, c->ws.cond_part) + i : nullptr;
            HIPCHK(launch_cfl(c->nd, fp64(c), a, s));
        }
    } else {
        a.leaves = dptr<int32_t>(c, c->ws.leaves);
        a.nleaves = c->nleaves;
        a.part = dptr<double>(c, c->ws.cfl_part);
        a.cpart = cond ? dptr<double>(c, c->ws.cond_part) : nullptr;
        HIPCHK(launch_cfl(c->nd, fp64(c), a, s));
    }
    return run_dt(c, dt_out, s, dt_int);
}

// after a restriction that formed the parts of every leaf with a parent:
// the parts of the leaves without one, then the dt records into dt_int
// whether the 2-D LF update forms the next cycle's CFL maxima of the leaves
// without parent that no reflux changes (map_launch::cfl_in_update); the
// automatic rule takes batched launches over at least 4 leaves per CU (a
// launch per block runs each update alone, latency-bound)
bool cfl_in_update(const map_ctx *c)
{
    if (c->nd != 2 || c->p.scheme != MAP_LF)
        return false;
    if (c->cfl_in_update >= 0)
        return c->cfl_in_update == 1;
    return c->launch_mode == MAP_LAUNCH_BATCHED && c->nleaves >= 4 * c->ncu;
}

// the CFL maxima of the leaves without parent that neither the restriction
// nor the update formed, then the dt records
map_status run_cfl_rest(map_ctx *c, const void *U, hipStream_t s, map_dt *dt_int)
{
    const bool fused = cfl_in_update(c);
    const size_t n = fused ? c->orphans_rest.size() : c->orphans.size();
    if (n > 0) {
        CflArgs a{};
        a.U = U;
        a.cnt = dptr<unsigned long long>(c, c->ws.counters);
        a.gamma = c->p.gamma;
        a.leaves = dptr<int32_t>(c, fused ? c->ws.orphans_rest : c->ws.orphans);
        a.nleaves = (int)n;
        a.part = dptr<double>(c, c->ws.cfl_part);
        a.part_idx = dptr<int32_t>(c, fused ? c->ws.orphan_rest_idx : c->ws.orphan_idx);
        HIPCHK(launch_cfl(c->nd, fp64(c), a, s));
    }
    return run_dt(c, nullptr, s, dt_int);
}

// one launch of the block-update kernel of the scheme (for WENO: one stage)
map_status run_step_kernel(map_ctx *c, int sch, const void *Uin, void *Uout, const void *Ubase,
                           const map_dt *dt, hipStream_t s, bool cfl_next = false)
{
    StepArgs a{};
    a.Uin = Uin;
    a.Uout = Uout;
    a.Ubase = Ubase;
    a.blk = dptr<BlockRec>(c, c->ws.blocks);
    a.dt = dt;
    a.lvl_dx = dptr<double>(c, c->ws.lvl_dx);
    a.fbidx = dptr<int32_t>(c, c->ws.fbidx);
    a.desc = dptr<Desc>(c, c->ws.desc);
    a.fbuf = c->wsp + c->ws.fbuf;
    a.cnt = dptr<unsigned long long>(c, c->ws.counters);
    a.gamma = c->p.gamma;
    a.eta = c->p.eta;
    a.eglm = c->p.eglm_sources;
    a.limiter = c->p.limiter;
    a.riemann = c->p.riemann;
    a.shape = c->step_shape;
    a.cfl_on = cfl_next && cfl_in_update(c);
    a.cfl_leaf = dptr<int32_t>(c, c->ws.cfl_leaf);
    a.cfl_part = dptr<double>(c, c->ws.cfl_part);
    const bool resist = c->p.eta > 0.0;
    auto launch = [&](const StepArgs &x, int grid) -> hipError_t {
        if (c->p.scheme == MAP_MMC)
            return launch_step_mmc(c->nd, fp64(c), x, 0.0, grid, s);
        if (c->nd == 3)
            return launch_step3(fp64(c), resist, sch, x, grid, s);
        return launch_step2(fp64(c), resist, sch, x, grid, s);
    };
    const int bpw = step_blocks_per_group(c->nd, c->p.scheme, c->step_shape);
    if (c->launch_mode == MAP_LAUNCH_PER_BLOCK) {
        for (int i = 0; i < c->nleaves; i++) {
            a.leaves = dptr<int32_t>(c, c->ws.leaves) + i;
            a.nleaves = 1;
            a.nitems = 1;
            HIPCHK(launch(a, 1));
        }
    } else {
        a.leaves = dptr<int32_t>(c, c->ws.leaves);
        a.nleaves = c->nleaves;
        a.nitems = (c->nleaves + bpw - 1) / bpw;
        HIPCHK(launch(a, c->grid_step));
    }
    return MAP_OK;
}

void *shadow(map_ctx *c);

// one update of every leaf from Uin to Uout.  WENO (Sec. 3.3): stage 1 into
// the shadow state, restriction and the ghosts the next stage reads from a
// block's own tile on it, stage 2 from the shadow with u^n = Uin; Uout may
// be Uin (stage 2 reads u^n only at the cell it writes)
map_status run_step(map_ctx *c, const void *Uin, void *Uout, const map_dt *dt, hipStream_t s,
                    bool cfl_next = false)
{
    if (c->p.scheme != MAP_WENO)
        return run_step_kernel(c, SCH_LF, Uin, Uout, nullptr, dt, s, cfl_next);
    map_status st;
    void *S1 = shadow(c);
    if ((st = run_step_kernel(c, SCH_WENO1, Uin, S1, nullptr, dt, s)) != MAP_OK)
        return st;
    if ((st = run_restrict(c, S1, s)) != MAP_OK)
        return st;
    if ((st = run_fill(c, S1, s, false)) != MAP_OK)
        return st;
    return run_step_kernel(c, SCH_WENO2, S1, Uout, Uin, dt, s);
}

map_status run_reflux(map_ctx *c, void *U, const map_dt *dt, hipStream_t s, int eonly_sub = -1)
{
    if (c->reflux_slots.empty())
        return MAP_OK;
    RefluxArgs a{};
    a.eonly = eonly_sub >= 0;
    a.sub = eonly_sub;
    a.nsims = (int)c->sims.size();
    a.U = U;
    a.slots = dptr<int32_t>(c, c->ws.reflux_slots);
    a.start = dptr<int32_t>(c, c->ws.reflux_start);
    a.recs = dptr<RefluxRec>(c, c->ws.reflux_recs);
    a.blk = dptr<BlockRec>(c, c->ws.blocks);
    a.dt = dt;
    a.lvl_dx = dptr<double>(c, c->ws.lvl_dx);
    a.fbuf = c->wsp + c->ws.fbuf;
    a.nitems = (int)c->reflux_slots.size();
    HIPCHK(launch_reflux(c->nd, fp64(c), a, s));
    return MAP_OK;
}

// the conduction subcycle of one step (Sec. 3.4, Fig. 1) with the records
// in dt (the device copy the kernels read); `scratch` is a whole state buffer
// whose contents are dead (its energy plane takes the new energy):
// cond_max_sub sub-steps are
// launched, and every pass skips the blocks of simulations whose own count
// nsub is smaller, so the launch sequence does not depend on device data
// (a captured graph replays it).  Each sub-step: the energy update into the
// scratch, commit, then reflux, restriction, exchange and prolongation of the
// energy alone.
map_status run_conduct(map_ctx *c, void *U, void *scratch, const map_dt *dt, hipStream_t s)
{
    if (c->p.cond_mode == MAP_COND_OFF)
        return MAP_OK;
    map_status st;
    CondArgs a{};
    a.U = U;
    a.S = scratch;
    a.blk = dptr<BlockRec>(c, c->ws.blocks);
    a.desc = dptr<Desc>(c, c->ws.desc);
    a.dt = dt;
    a.lvl_dx = dptr<double>(c, c->ws.lvl_dx);
    a.fbidx = dptr<int32_t>(c, c->ws.fbidx);
    a.fbuf = c->wsp + c->ws.fbuf;
    a.gamma = c->p.gamma;
    a.kappa0 = c->p.kappa0;
    a.khalf = (int)(2.0 * c->p.kappa_exp + 0.5);
    a.mode = c->p.cond_mode;
    a.list = dptr<int32_t>(c, c->ws.leaves);
    a.nitems = c->nleaves;
    a.nsims = (int)c->sims.size();
    for (int i = 0; i < c->p.cond_max_sub; i++) {
        a.sub = i;
        HIPCHK(launch_conduct(c->nd, fp64(c), a, s));
        HIPCHK(launch_cond_commit(c->nd, fp64(c), a, s));
        if ((st = run_reflux(c, U, dt, s, i)) != MAP_OK)
            return st;
        if ((st = run_restrict(c, U, s, i, false, dt)) != MAP_OK)
            return st;
        if ((st = run_fill(c, U, s, false, i, dt)) != MAP_OK)
            return st;
    }
    return MAP_OK;
}

// one cycle from Uin to Uout (Fig. 1) with the dt records `dt` (formed here
// from Uin if need_cfl): update of every leaf, reflux, restriction, the
// ghosts the next update reads from its own tile, and the conduction
// subcycle when it is on (its scratch: Uin, dead after the update, or the
// shadow when the cycle runs in place).  With `next`, the next cycle's dt
// records are formed into `next` on the way: the restriction takes the CFL
// maxima of the leaves with a parent from the values it reads (final after
// reflux), the 2-D LF update those of the leaves without one that no reflux
// changes (from the values it writes), a small pass the rest.
map_status run_cycle(map_ctx *c, const void *Uin, void *Uout, hipStream_t s, map_dt *dt,
                     bool need_cfl, map_dt *next)
{
    map_status st;
    if (need_cfl && (st = run_cfl(c, Uin, nullptr, s, dt)) != MAP_OK)
        return st;
    if ((st = run_step(c, Uin, Uout, dt, s, next != nullptr)) != MAP_OK)
        return st;
    if ((st = run_reflux(c, Uout, dt, s)) != MAP_OK)
        return st;
    if ((st = run_restrict(c, Uout, s, -1, next != nullptr)) != MAP_OK)
        return st;
    if ((st = run_fill(c, Uout, s, false)) != MAP_OK)
        return st;
    if (next && (st = run_cfl_rest(c, Uout, s, next)) != MAP_OK)
        return st;
    void *scratch = Uin != Uout ? const_cast<void *>(Uin) : shadow(c);
    return run_conduct(c, Uout, scratch, dt, s);
}

// the next cycle's dt can come from this one only if the leaf interiors are
// final after the restriction: not with the conduction subcycle, which
// changes the energy after the fill
bool chain_dt(const map_ctx *c) { return c->p.cond_mode == MAP_COND_OFF; }

size_t state_bytes(const map_ctx *c) { return (size_t)c->nslots * NV * c->tile * c->word; }

void *shadow(map_ctx *c) { return c->wsp + c->ws.shadow; }

// n cycles alternating between U and the workspace's shadow state; an odd
// count ends with one copy of the shadow back into U.  WENO cycles run in
// place (the shadow holds the Runge-Kutta stage).  The first cycle forms its
// dt records; each later one takes those the cycle before formed, the two
// alternating between the two record buffers.
map_status run_cycles(map_ctx *c, void *U, int n, hipStream_t s)
{
    map_status st;
    const bool chain = chain_dt(c);
    const size_t off[2] = {c->ws.dt, c->ws.dt2};
    int cur = 0;
    bool need = true;
    void *S2 = shadow(c);
    for (int i = 0; i < n; i++) {
        void *in = U, *out = U;
        if (c->p.scheme != MAP_WENO) {
            const bool even = (i & 1) == 0;
            in = even ? U : S2;
            out = even ? S2 : U;
        }
        map_dt *next = chain && i + 1 < n ? dptr<map_dt>(c, off[cur ^ 1]) : nullptr;
        if ((st = run_cycle(c, in, out, s, dptr<map_dt>(c, off[cur]), need, next)) != MAP_OK)
            return st;
        c->last_dt = off[cur];
        if (next) {
            cur ^= 1;
            need = false;
        } else {
            need = true;
        }
    }
    if (c->p.scheme != MAP_WENO && (n & 1))
        HIPCHK(hipMemcpyAsync(U, S2, state_bytes(c), hipMemcpyDeviceToDevice, s));
    return MAP_OK;
}

void drop_graph(map_ctx *c)
{
    if (c->graph_exec) {
        hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(c->graph_exec));
        c->graph_exec = nullptr;
    }
    if (c->graph_exec2) {
        hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(c->graph_exec2));
        c->graph_exec2 = nullptr;
    }
    c->graph_U = nullptr;
}

}  // namespace

// error reporting for the host tree edit (regrid.cpp)
map_status regrid_fail(map_status st, const std::string &msg) { return fail(st, msg); }

extern "C" {

const char *map_last_error(void) { return g_err.c_str(); }

map_status map_init_blocks(map_ctx **ctx, const map_params *params, int nsims,
                           const map_sim_desc *sims, int nblocks, const map_block_key *keys)
{
    if (!ctx)
        return fail(MAP_EINVAL, "null ctx pointer");
    *ctx = nullptr;
    map_ctx *c = new (std::nothrow) map_ctx();
    if (!c)
        return fail(MAP_EINVAL, "out of host memory");
    std::string err;
    map_status st;
    try {
        st = map_plan_build(c, params, nsims, sims, nblocks, keys, err);
    } catch (const std::exception &e) {
        st = MAP_EINVAL;
        err = std::string("host exception: ") + e.what();
    }
    if (st != MAP_OK) {
        delete c;
        return fail(st, err);
    }
    *ctx = c;
    return MAP_OK;
}

map_status map_query(const map_ctx *c, map_sizes *sz, int32_t *slot_of_key)
{
    if (!c || !sz)
        return fail(MAP_EINVAL, "null argument");
    sz->state_bytes = state_bytes(c);
    sz->workspace_bytes = c->ws.total;
    sz->nblocks = c->nslots;
    sz->nleaves = c->nleaves;
    sz->nsims = (int)c->sims.size();
    sz->max_level = c->lmax;
    sz->tile_cells = c->tile;
    sz->nvar = NV;
    sz->n_prolong_items = (int)c->prolong_list.size();
    sz->n_reflux_blocks = (int)c->reflux_slots.size();
    sz->n_face_buffers = c->nfb;
    if (slot_of_key)
        std::memcpy(slot_of_key, c->slot_of_key.data(), sizeof(int32_t) * c->nslots);
    return MAP_OK;
}

/* Ghost source of every (input key, direction): the input index of the
 * same-level block whose cells are copied, -1 where ghosts are prolongated
 * from the parent, -2 for the block itself (direction 0) or unused
 * directions (dz != 0 in 2-D).  neigh[nblocks][27], direction index
 * (dz+1)*9 + (dy+1)*3 + (dx+1).  Host only. */
map_status map_neighbors(const map_ctx *c, int32_t *neigh)
{
    if (!c || !neigh)
        return fail(MAP_EINVAL, "null argument");
    std::vector<int32_t> key_of_slot(c->nslots);
    for (int i = 0; i < c->nslots; i++)
        key_of_slot[c->slot_of_key[i]] = i;
    for (int i = 0; i < c->nslots; i++) {
        int s = c->slot_of_key[i];
        for (int d = 0; d < NDIR; d++) {
            int src = c->desc[(size_t)s * NDIR + d].src;
            neigh[(size_t)i * NDIR + d] = src >= 0 ? key_of_slot[src] : src;
        }
    }
    return MAP_OK;
}

map_status map_fill_selection(const map_ctx *c, int cap, int32_t *parent, uint32_t *dirs,
                              int32_t *box, int *count)
{
    if (!c || !count || cap < 0 || (cap > 0 && (!parent || !dirs || !box)))
        return fail(MAP_EINVAL, "null argument or negative capacity");
    std::vector<int32_t> key_of_slot(c->nslots);
    for (int i = 0; i < c->nslots; i++)
        key_of_slot[c->slot_of_key[i]] = i;
    const int n = (int)c->frame_list.size();
    for (int i = 0; i < n && i < cap; i++) {
        const FrameSel &f = c->frame_sel[i];
        parent[i] = key_of_slot[c->frame_list[i]];
        dirs[i] = f.dirs;
        for (int d = 0; d < 3; d++) {
            box[(size_t)i * 6 + d] = f.lo[d];
            box[(size_t)i * 6 + 3 + d] = f.hi[d];
        }
    }
    *count = n;
    return MAP_OK;
}

map_status map_bind_workspace(map_ctx *c, void *ws, size_t bytes, void *stream)
{
    if (!c || !ws)
        return fail(MAP_EINVAL, "null argument");
    if (bytes < c->ws.total)
        return fail(MAP_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes, need " +
                                    std::to_string(c->ws.total));
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(MAP_EINVAL, "workspace must be 256-byte aligned");
    drop_graph(c);
    c->wsp = static_cast<char *>(ws);
    hipStream_t s = S(stream);
    auto up = [&](size_t off, const void *src, size_t n) -> hipError_t {
        if (n == 0)
            return hipSuccess;
        return hipMemcpyAsync(c->wsp + off, src, n, hipMemcpyHostToDevice, s);
    };
    HIPCHK(up(c->ws.blocks, c->blk.data(), c->blk.size() * sizeof(BlockRec)));
    HIPCHK(up(c->ws.desc, c->desc.data(), c->desc.size() * sizeof(Desc)));
    HIPCHK(up(c->ws.parent, c->parent.data(), c->parent.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.children, c->children.data(), c->children.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.fbidx, c->fbidx.data(), c->fbidx.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.leaves, c->leaves.data(), c->leaves.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.leaf_of, c->leaf_of.data(), c->leaf_of.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.orphans, c->orphans.data(), c->orphans.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.orphan_idx, c->orphan_idx.data(), c->orphan_idx.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.cfl_leaf, c->cfl_leaf.data(), c->cfl_leaf.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.orphans_rest, c->orphans_rest.data(), c->orphans_rest.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.orphan_rest_idx, c->orphan_rest_idx.data(),
              c->orphan_rest_idx.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.restrict_list, c->restrict_list.data(), c->restrict_list.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.prolong_list, c->prolong_list.data(), c->prolong_list.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.prolong_mask, c->prolong_mask.data(), c->prolong_mask.size() * sizeof(uint32_t)));
    HIPCHK(up(c->ws.frame_list, c->frame_list.data(), c->frame_list.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.frame_sel, c->frame_sel.data(), c->frame_sel.size() * sizeof(FrameSel)));
    HIPCHK(up(c->ws.reflux_slots, c->reflux_slots.data(), c->reflux_slots.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.reflux_start, c->reflux_start.data(), c->reflux_start.size() * sizeof(int32_t)));
    HIPCHK(up(c->ws.reflux_recs, c->reflux_recs.data(), c->reflux_recs.size() * sizeof(RefluxRec)));
    HIPCHK(up(c->ws.sims, c->simrec.data(), c->simrec.size() * sizeof(SimRec)));
    HIPCHK(up(c->ws.lvl_dx, c->lvl_dx.data(), c->lvl_dx.size() * sizeof(double)));
    HIPCHK(launch_clear_u64(dptr<unsigned long long>(c, c->ws.counters), 4, s));
    // the host vectors above are pageable: finish the copies before returning
    HIPCHK(hipStreamSynchronize(s));
    c->last_dt = c->ws.dt;
    {
        // the static scratch's address on this device, once per device
        double *sp = nullptr;
        map_status sst = scratch_of_current_device(&sp);
        if (sst != MAP_OK)
            return sst;
    }
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        ncu > 0)
        c->ncu = ncu;
    c->bound = true;
    return MAP_OK;
}

map_status map_prim_to_cons(map_ctx *c, void *U, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U)
        return fail(MAP_EINVAL, "null U");
    HIPCHK(launch_prim_to_cons(fp64(c), U, (size_t)c->nslots, c->tile, c->p.gamma, S(stream)));
    return MAP_OK;
}

map_status map_fill_ghosts(map_ctx *c, void *U, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U)
        return fail(MAP_EINVAL, "null U");
    return run_fill(c, U, S(stream), true);
}

map_status map_restrict(map_ctx *c, void *U, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U)
        return fail(MAP_EINVAL, "null U");
    return run_restrict(c, U, S(stream));
}

map_status map_prolong(map_ctx *c, void *U, const int32_t *slots_dev, int n, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U || (n > 0 && !slots_dev) || n < 0)
        return fail(MAP_EINVAL, "null U or slot list");
    FillArgs a{};
    a.U = U;
    a.blk = dptr<BlockRec>(c, c->ws.blocks);
    a.parent = dptr<int32_t>(c, c->ws.parent);
    a.list = slots_dev;
    a.nitems = n;
    HIPCHK(launch_prolong_blocks(c->nd, fp64(c), a, S(stream)));
    return MAP_OK;
}

map_status map_cfl_dt(map_ctx *c, const void *U, map_dt *dt_dev, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U)
        return fail(MAP_EINVAL, "null U");
    c->last_dt = c->ws.dt;
    return run_cfl(c, U, dt_dev, S(stream));
}

map_status map_step(map_ctx *c, const void *Uin, void *Uout, const map_dt *dt_dev, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!Uin || !Uout || !dt_dev)
        return fail(MAP_EINVAL, "null U or dt");
    {
        const char *i0 = static_cast<const char *>(Uin), *o0 = static_cast<const char *>(Uout);
        const size_t nb = state_bytes(c);
        const bool same = c->p.scheme == MAP_WENO && i0 == o0;
        if (!same && i0 < o0 + nb && o0 < i0 + nb)
            return fail(MAP_EINVAL, "Uout overlaps Uin (the update reads neighbour cells of Uin)");
        const char *w0 = c->wsp;
        if (o0 < w0 + c->ws.total && w0 < o0 + nb)
            return fail(MAP_EINVAL, "Uout overlaps the bound workspace");
    }
    return run_step(c, Uin, Uout, dt_dev, S(stream));
}

map_status map_reflux(map_ctx *c, void *U, const map_dt *dt_dev, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U || !dt_dev)
        return fail(MAP_EINVAL, "null U or dt");
    return run_reflux(c, U, dt_dev, S(stream));
}

map_status map_conduct(map_ctx *c, void *U, const map_dt *dt_dev, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U || !dt_dev)
        return fail(MAP_EINVAL, "null U or dt");
    const char *u0 = static_cast<const char *>(U), *w0 = c->wsp;
    if (u0 < w0 + c->ws.total && w0 < u0 + state_bytes(c))
        return fail(MAP_EINVAL, "U overlaps the bound workspace");
    return run_conduct(c, U, shadow(c), dt_dev, S(stream));
}

// totals of the leaves with the per-leaf partial sums in `part`
// (nleaves x NV doubles, every entry written before it is read)
map_status run_totals(map_ctx *c, const void *U, double *totals_dev, double *part, hipStream_t s)
{
    TotalsArgs a{};
    a.U = U;
    a.leaves = dptr<int32_t>(c, c->ws.leaves);
    a.nleaves = c->nleaves;
    a.blk = dptr<BlockRec>(c, c->ws.blocks);
    a.lvl_dx = dptr<double>(c, c->ws.lvl_dx);
    a.part = part;
    a.sims = dptr<SimRec>(c, c->ws.sims);
    a.out = totals_dev;
    a.nsims = (int)c->sims.size();
    a.ndim = c->nd;
    HIPCHK(launch_totals(c->nd, fp64(c), a, s));
    return MAP_OK;
}

map_status map_totals(map_ctx *c, const void *U, double *totals_dev, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U || !totals_dev)
        return fail(MAP_EINVAL, "null U or output");
    return run_totals(c, U, totals_dev, dptr<double>(c, c->ws.tot_part), S(stream));
}

map_status map_totals_static(map_ctx *c, const void *U, double *totals_dev, void *stream)
{
    if (!c)
        return fail(MAP_EINVAL, "null context");
    const size_t need = (size_t)c->nleaves * NV;
    if (need > (size_t)MAP_STATIC_SCRATCH_DOUBLES)
        return fail(MAP_EINVAL, std::to_string(c->nleaves) + " leaves need " +
                                    std::to_string(need) + " doubles of scratch; the static "
                                    "scratch holds " + std::to_string(MAP_STATIC_SCRATCH_DOUBLES) +
                                    " (" + std::to_string(MAP_STATIC_SCRATCH_DOUBLES / NV) +
                                    " leaves)");
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U || !totals_dev)
        return fail(MAP_EINVAL, "null U or output");
    double *part = nullptr;
    if ((st = scratch_of_current_device(&part)) != MAP_OK)
        return st;
    return run_totals(c, U, totals_dev, part, S(stream));
}

map_status map_status_flags(map_ctx *c, uint64_t counters[4], void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!counters)
        return fail(MAP_EINVAL, "null counters");
    hipStream_t s = S(stream);
    unsigned long long h[4];
    HIPCHK(hipMemcpyAsync(h, c->wsp + c->ws.counters, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(launch_clear_u64(dptr<unsigned long long>(c, c->ws.counters), 4, s));
    for (int i = 0; i < 4; i++)
        counters[i] = h[i];
    if (h[3])
        return fail(MAP_ENONFINITE, std::to_string(h[3]) + " non-finite cells");
    if (h[2])
        return fail(MAP_ENEGPRESSURE, std::to_string(h[2]) + " cells with rho <= 0 or p <= 0");
    return MAP_OK;
}

map_status map_advance(map_ctx *c, void *U, map_dt *dt_dev, int nsteps, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U || nsteps < 0)
        return fail(MAP_EINVAL, "null U or negative step count");
    hipStream_t s = S(stream);
    if ((st = run_cycles(c, U, nsteps, s)) != MAP_OK)
        return st;
    if (dt_dev && nsteps > 0)
        HIPCHK(hipMemcpyAsync(dt_dev, c->wsp + c->last_dt, sizeof(map_dt) * c->sims.size(),
                              hipMemcpyDeviceToDevice, s));
    return MAP_OK;
}

map_status map_graph_run(map_ctx *c, void *U, map_dt *dt_dev, int nsteps, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U || nsteps < 0)
        return fail(MAP_EINVAL, "null U or negative step count");
    hipStream_t s = S(stream);
    const bool chain = chain_dt(c);
    if (!c->graph_exec || c->graph_U != U) {
        drop_graph(c);
        if (!c->cap_stream) {
            hipStream_t cs;
            HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            c->cap_stream = cs;
        }
        hipStream_t cs = S(c->cap_stream);
        // two cycles, U -> shadow -> U (WENO: U -> U twice).  With chained
        // dt records: the first pair of a run forms its first records, each
        // cycle forms the next one's (the second cycle's for the next pair),
        // and the later pairs start from those; otherwise every cycle forms
        // its own.
        void *mid = c->p.scheme == MAP_WENO ? U : shadow(c);
        map_dt *D0 = dptr<map_dt>(c, c->ws.dt), *D1 = dptr<map_dt>(c, c->ws.dt2);
        auto capture = [&](bool first, void **out) -> map_status {
            HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
            map_status r = chain ? run_cycle(c, U, mid, cs, D0, first, D1)
                                 : run_cycle(c, U, mid, cs, D0, true, nullptr);
            if (r == MAP_OK)
                r = chain ? run_cycle(c, mid, U, cs, D1, false, D0)
                          : run_cycle(c, mid, U, cs, D0, true, nullptr);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(cs, &g);
            if (r != MAP_OK) {
                if (g)
                    hipGraphDestroy(g);
                return r;
            }
            if (e != hipSuccess)
                return fail(MAP_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            hipGraphExec_t ex = nullptr;
            e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (e != hipSuccess)
                return fail(MAP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            *out = ex;
            return MAP_OK;
        };
        if ((st = capture(true, &c->graph_exec)) != MAP_OK)
            return st;
        if (chain && (st = capture(false, &c->graph_exec2)) != MAP_OK) {
            drop_graph(c);
            return st;
        }
        c->graph_U = U;
    }
    for (int i = 0; i + 1 < nsteps; i += 2) {
        void *ex = chain && i > 0 ? c->graph_exec2 : c->graph_exec;
        HIPCHK(hipGraphLaunch(reinterpret_cast<hipGraphExec_t>(ex), s));
        c->last_dt = chain ? c->ws.dt2 : c->ws.dt;
    }
    if ((nsteps & 1) && (st = run_cycles(c, U, 1, s)) != MAP_OK)
        return st;
    if (dt_dev && nsteps > 0)
        HIPCHK(hipMemcpyAsync(dt_dev, c->wsp + c->last_dt, sizeof(map_dt) * c->sims.size(),
                              hipMemcpyDeviceToDevice, s));
    return MAP_OK;
}

map_status map_set_launch(map_ctx *c, int mode, int grid_step, int grid_fill)
{
    if (!c)
        return fail(MAP_EINVAL, "null context");
    if (mode != MAP_LAUNCH_BATCHED && mode != MAP_LAUNCH_PER_BLOCK)
        return fail(MAP_EINVAL, "unknown launch mode");
    if (grid_step < 0 || grid_fill < 0)
        return fail(MAP_EINVAL, "negative grid size");
    drop_graph(c);
    c->launch_mode = mode;
    c->grid_step = grid_step;
    c->grid_fill = grid_fill;
    return MAP_OK;
}

// whether the update of this context has a second workgroup shape
static bool has_step_shapes(const map_ctx *c)
{
    if (c->p.scheme == MAP_MMC)
        return false;
    return c->nd == 2 || c->p.precision == MAP_FP32_MIXED;
}

map_status map_get_launch(const map_ctx *c, map_launch *out)
{
    if (!c || !out)
        return fail(MAP_EINVAL, "null argument");
    out->mode = c->launch_mode;
    out->grid_step = c->grid_step;
    out->grid_fill = c->grid_fill;
    out->step_shape = c->step_shape;
    out->restrict_split = c->restrict_split >= 0 ? c->restrict_split : c->ncu;
    out->step_blocks_per_group = step_blocks_per_group(c->nd, c->p.scheme, c->step_shape);
    out->cfl_in_update = c->cfl_in_update;
    out->cfl_in_update_on = cfl_in_update(c) ? 1 : 0;
    return MAP_OK;
}

map_status map_set_launch_config(map_ctx *c, const map_launch *in)
{
    if (!c || !in)
        return fail(MAP_EINVAL, "null argument");
    if (in->step_shape < 0 || in->step_shape > 1 || (in->step_shape == 1 && !has_step_shapes(c)))
        return fail(MAP_EINVAL, "step_shape 1 exists for 2-D LF/WENO and 3-D FP32 LF/WENO only");
    if (in->restrict_split < -1)
        return fail(MAP_EINVAL, "restrict_split below -1");
    if (in->cfl_in_update < -1 || in->cfl_in_update > 1)
        return fail(MAP_EINVAL, "cfl_in_update must be -1, 0 or 1");
    map_status st = map_set_launch(c, in->mode, in->grid_step, in->grid_fill);
    if (st)
        return st;
    c->step_shape = in->step_shape;
    c->restrict_split = in->restrict_split;
    c->cfl_in_update = in->cfl_in_update;
    return MAP_OK;
}

map_status map_autotune(map_ctx *c, void *U, int *chosen, void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U)
        return fail(MAP_EINVAL, "null U");
    hipStream_t s = S(stream);
    const int saved_mode = c->launch_mode;
    c->launch_mode = MAP_LAUNCH_BATCHED;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    map_dt *dt = dptr<map_dt>(c, c->ws.dt);
    if ((st = run_cfl(c, U, nullptr, s)) != MAP_OK)
        return st;
    // one untimed launch (the candidate's code and data warm), then the
    // best of five
    auto time_it = [&](auto &&fn) -> float {
        if (fn() != MAP_OK)
            return 1e30f;
        float best = 1e30f;
        for (int r = 0; r < 5; r++) {
            hipEventRecord(e0, s);
            if (fn() != MAP_OK)
                return 1e30f;
            hipEventRecord(e1, s);
            hipEventSynchronize(e1);
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, ms);
        }
        return best;
    };
    // a candidate replaces the current choice only when it is faster by more
    // than the run-to-run spread of these timings (0.5 %), so that near-ties
    // keep the first candidate tried, the simplest shape
    auto faster = [](float t, float best) { return t < 0.995f * best; };
    // persistent grids: multiples of the compute units below the item count,
    // and one workgroup per work item (0)
    auto grids = [&](int nitems) {
        std::vector<int> g = {0};
        for (int m : {1, 2, 4, 8, 16})
            if (c->ncu * m < nitems)
                g.push_back(c->ncu * m);
        return g;
    };
    // the update: workgroup shape x persistent grid
    int best_shape = 0, best_step = 0;
    float best_t = 1e30f;
    const int nshapes = has_step_shapes(c) ? 2 : 1;
    for (int shape = 0; shape < nshapes; shape++) {
        c->step_shape = shape;
        const int bpw = step_blocks_per_group(c->nd, c->p.scheme, shape);
        for (int g : grids((c->nleaves + bpw - 1) / bpw)) {
            c->grid_step = g;
            const int sch = c->p.scheme == MAP_WENO ? SCH_WENO1 : SCH_LF;
            float t = time_it([&] { return run_step_kernel(c, sch, U, shadow(c), nullptr, dt, s); });
            if (faster(t, best_t)) {
                best_t = t;
                best_shape = shape;
                best_step = g;
            }
        }
    }
    c->step_shape = best_shape;
    c->grid_step = best_step;
    // the parent-frame copies of the cycle's fill
    const int fbpw = fill_blocks_per_group(c->nd);
    int best_fill = 0;
    best_t = 1e30f;
    for (int g : grids(((int)c->frame_list.size() + fbpw - 1) / fbpw)) {
        c->grid_fill = g;
        float t = time_it([&] { return run_fill(c, U, s, false); });
        if (faster(t, best_t)) {
            best_t = t;
            best_fill = g;
        }
    }
    c->grid_fill = best_fill;
    // restriction: below how many parents a level takes one workgroup per
    // child (it rewrites the parents' interiors with the same values)
    int best_split = c->ncu;
    if (c->lmax > 1) {
        best_t = 1e30f;
        for (int sp : {0, c->ncu / 2, c->ncu, 2 * c->ncu, 4 * c->ncu, 1 << 30}) {
            c->restrict_split = sp;
            float t = time_it([&] { return run_restrict(c, U, s); });
            if (faster(t, best_t)) {
                best_t = t;
                best_split = sp;
            }
        }
    }
    c->restrict_split = best_split;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    drop_graph(c);
    c->launch_mode = saved_mode;
    if (chosen) {
        chosen[0] = best_step;
        chosen[1] = best_fill;
    }
    return MAP_OK;
}

map_status map_estimate(map_ctx *c, const void *U, const map_estimator *est, double *err_dev,
                        void *stream)
{
    map_status st = need_bound(c);
    if (st)
        return st;
    if (!U || !est || !err_dev)
        return fail(MAP_EINVAL, "null U, estimator or output");
    if (est->ncrit < 1 || est->ncrit > 4)
        return fail(MAP_EINVAL, "ncrit must be 1..4");
    for (int i = 0; i < est->ncrit; i++) {
        if (est->mode[i] != MAP_EST_VAR && est->mode[i] != MAP_EST_BMAG)
            return fail(MAP_EINVAL, "unknown estimator mode");
        if (est->mode[i] == MAP_EST_VAR && (est->var[i] < 0 || est->var[i] >= NV))
            return fail(MAP_EINVAL, "estimator variable out of range");
    }
    EstArgs a{};
    a.U = U;
    a.desc = dptr<Desc>(c, c->ws.desc);
    a.blk = dptr<BlockRec>(c, c->ws.blocks);
    a.err = err_dev;
    a.nslots = c->nslots;
    a.est = *est;
    HIPCHK(launch_estimate(c->nd, fp64(c), a, S(stream)));
    return MAP_OK;
}

map_status map_remap(map_ctx *dst, void *Ud, const map_ctx *src, const void *Us, void *stream)
{
    map_status st = need_bound(dst);
    if (st)
        return st;
    if (!src || !src->bound)
        return fail(MAP_ESTATE, "source context not bound");
    if (!Ud || !Us)
        return fail(MAP_EINVAL, "null state");
    if (src->nd != dst->nd || src->p.precision != dst->p.precision ||
        src->sims.size() != dst->sims.size() ||
        std::memcmp(src->sims.data(), dst->sims.data(), sizeof(map_sim_desc) * src->sims.size()))
        return fail(MAP_EINVAL, "contexts differ in dimension, precision or simulations");
    KeyMap src_slot(src->nslots);
    auto pack = [](const map_block_key &k) {
        return ((uint64_t)k.sim << 47) | ((uint64_t)k.level << 42) | ((uint64_t)k.ix << 28) |
               ((uint64_t)k.iy << 14) | (uint64_t)k.iz;
    };
    for (int s = 0; s < src->nslots; s++)
        src_slot.insert(pack(src->key[s]), s);
    dst->remap_src.assign(dst->nslots, -1);
    dst->remap_new.clear();
    for (int s = 0; s < dst->nslots; s++) {
        const int from = src_slot.find(pack(dst->key[s]));
        if (from >= 0) {
            dst->remap_src[s] = from;
            continue;
        }
        const int p = dst->parent[s];
        if (p < 0 || !src_slot.contains(pack(dst->key[p])))
            return fail(MAP_ETREE, "a new block's parent is not in the source tree");
        dst->remap_new.push_back(s);
    }
    hipStream_t s = S(stream);
    HIPCHK(hipMemcpyAsync(dst->wsp + dst->ws.remap, dst->remap_src.data(),
                          sizeof(int32_t) * dst->nslots, hipMemcpyHostToDevice, s));
    if (!dst->remap_new.empty())
        HIPCHK(hipMemcpyAsync(dst->wsp + dst->ws.newlist, dst->remap_new.data(),
                              sizeof(int32_t) * dst->remap_new.size(), hipMemcpyHostToDevice, s));
    RemapArgs r{};
    r.Udst = Ud;
    r.Usrc = Us;
    r.map = dptr<int32_t>(dst, dst->ws.remap);
    r.tile_bytes = (size_t)NV * dst->tile * dst->word;
    r.nslots = dst->nslots;
    HIPCHK(launch_remap_copy(r, s));
    // ghosts of the surviving blocks (the parents of new blocks are among
    // them), then the new blocks from their parents, then restriction and
    // a complete fill
    if ((st = run_fill(dst, Ud, s, true)) != MAP_OK)
        return st;
    if (!dst->remap_new.empty()) {
        FillArgs a{};
        a.U = Ud;
        a.blk = dptr<BlockRec>(dst, dst->ws.blocks);
        a.parent = dptr<int32_t>(dst, dst->ws.parent);
        a.list = dptr<int32_t>(dst, dst->ws.newlist);
        a.nitems = (int)dst->remap_new.size();
        HIPCHK(launch_prolong_blocks(dst->nd, fp64(dst), a, s));
    }
    if ((st = run_restrict(dst, Ud, s)) != MAP_OK)
        return st;
    if ((st = run_fill(dst, Ud, s, true)) != MAP_OK)
        return st;
    HIPCHK(hipStreamSynchronize(s));
    return MAP_OK;
}

void map_destroy(map_ctx *c)
{
    if (!c)
        return;
    drop_graph(c);
    if (c->cap_stream)
        hipStreamDestroy(S(c->cap_stream));
    delete c;
}

}  // extern "C"
