// plan.hpp -- host-side context: the validated block tree in Morton order and
// the tables the kernels read (the neighbour statistics of Sec. 4.2).
#pragma once

#include <string>
#include <vector>

#include "map_internal.hpp"

struct map_ctx {
    map_params p{};
    int nd = 2;
    int tile = 0;                          // padded cells per variable
    int nslots = 0, nleaves = 0, lmax = 1;
    std::vector<map_sim_desc> sims;
    std::vector<int32_t> slot_of_key;      // input index -> slot
    std::vector<map_block_key> key;        // by slot
    std::vector<mapk::BlockRec> blk;       // by slot
    std::vector<int32_t> parent;           // by slot, -1 at level 1
    std::vector<int32_t> children;         // [slot][8], -1 if none
    std::vector<mapk::Desc> desc;          // [slot][27]
    std::vector<int32_t> fbidx;            // [slot][6], -1 if none
    std::vector<int32_t> leaves;           // leaf slots in Morton order
    std::vector<int32_t> leaf_of;          // by slot: index in `leaves`, -1 for parents
    std::vector<int32_t> orphans;          // leaves without a parent (level 1), and
    std::vector<int32_t> orphan_idx;       // their indices in `leaves`
    std::vector<int32_t> cfl_leaf;         // by slot: index in `leaves` of a leaf without
                                           // parent whose next CFL maximum the 2-D LF
                                           // update can form (no reflux after it), else -1
    std::vector<int32_t> orphans_rest;     // the other leaves without parent, and their
    std::vector<int32_t> orphan_rest_idx;  // indices in `leaves`
    std::vector<mapk::SimRec> simrec;
    std::vector<double> lvl_dx;            // [sim][MAXL + 1][3]
    std::vector<int32_t> restrict_list;    // parent slots, grouped by level
    std::vector<int> restrict_off;         // [lmax + 1] offsets by level
    std::vector<int32_t> prolong_list;     // slots with prolongated ghosts, by level
    std::vector<int> prolong_off;          // [lmax + 2]
    std::vector<uint32_t> prolong_mask;    // per prolong_list entry: bit d set if ghost
                                           // direction d is prolongated
    std::vector<int32_t> frame_list;       // parents of prolong_list slots (their ghost
                                           // frames feed the prolongation), slot order
    std::vector<mapk::FrameSel> frame_sel; // per frame_list entry: the ghost cells the
                                           // prolongation stencil reads (a superset)
    std::vector<int32_t> reflux_slots;     // coarse leaves with reflux faces
    std::vector<int32_t> reflux_start;     // [n + 1] into reflux_recs
    std::vector<mapk::RefluxRec> reflux_recs;
    int nfb = 0;                           // face buffers

    // device binding
    mapk::WsLayout ws{};
    char *wsp = nullptr;
    bool bound = false;
    size_t word = 8;

    // launch configuration
    int launch_mode = MAP_LAUNCH_BATCHED;
    int grid_step = 0, grid_fill = 0;
    int step_shape = 0;        // workgroup shape of the update (StepArgs::shape)
    int restrict_split = -1;   // levels with fewer parents take one workgroup per child (-1: ncu)
    int cfl_in_update = -1;    // map_launch::cfl_in_update
    int ncu = 256;  // compute units of the bound device

    // map_remap: by slot, the source slot in the previous tree (-1: new
    // block), and the new blocks (host copies kept for the async upload)
    std::vector<int32_t> remap_src, remap_new;

    // captured cycles: the first pair of a run (it forms its first dt
    // records) and the pairs after it (they start from the records the pair
    // before formed during its last restriction)
    void *graph_exec = nullptr;   // hipGraphExec_t
    void *graph_exec2 = nullptr;  // hipGraphExec_t
    void *graph_U = nullptr;
    void *cap_stream = nullptr;  // hipStream_t used for capture
    size_t last_dt = 0;          // workspace offset of the last cycle's dt records

    size_t face_cells() const { return nd == 3 ? (size_t)mapk::NB * mapk::NB : (size_t)mapk::NB; }
};

// builds everything above except the device binding; returns MAP_OK,
// MAP_EINVAL or MAP_ETREE with a message in `err`
map_status map_plan_build(map_ctx *c, const map_params *p, int nsims, const map_sim_desc *sims,
                          int nblocks, const map_block_key *keys, std::string &err);
void map_plan_layout(map_ctx *c);
uint64_t map_morton3(uint32_t x, uint32_t y, uint32_t z);
