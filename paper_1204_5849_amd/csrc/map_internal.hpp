// map_internal.hpp -- layout constants and device-table records shared by the
// host runtime (plan.cpp, api.hip) and the kernels.  Product code only.
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/map.h"

namespace mapk {

constexpr int NB = 16;        // cells per block edge
constexpr int NG = 2;         // ghost layers
constexpr int PD = NB + 2 * NG;  // padded edge (20)
constexpr int NV = 9;         // rho, m_x, m_y, m_z, B_x, B_y, B_z, e, psi
constexpr int MAXL = 16;      // levels per simulation
constexpr int NDIR = 27;      // neighbour directions (3^3; 2-D uses the dz = 0 plane)
constexpr int CLAMP = 1024;   // descriptor offset code: source index = value - CLAMP

enum { RHO = 0, MX = 1, MY = 2, MZ = 3, BX = 4, BY = 5, BZ = 6, EN = 7, PSI = 8 };

// per-slot record: x = sim, y = level, z = child position bits (cx | cy<<1 | cz<<2),
// w = 1 for leaves
struct BlockRec {
    int sim, level, cpos, leaf;
};

// ghost descriptor of one (slot, direction): source slot (or -1: prolongate
// from the parent, -2: unused) and per-dimension source index rule
// (offset added to the ghost index, or CLAMP + fixed index)
struct Desc {
    int src, o0, o1, o2;
};

// the part of a parent's ghost frame that a fill by copies writes: ghost
// cells of the directions set in `dirs` inside the padded-cell box [lo, hi]
struct FrameSel {
    uint32_t dirs;
    int lo[3], hi[3];
    int pad;
};

// one coarse face next to finer leaves: dimension, side, face buffer of the
// coarse block and of the 2^(d-1) fine blocks, ordered by transverse halves
struct RefluxRec {
    int dim, side, fb_coarse, pad;
    int fb_fine[4];
};

struct SimRec {
    double dxmin;        // smallest leaf cell width of the simulation
    int leaf_lo, leaf_hi;  // range in the leaf list
};

// byte offsets of the tables inside the caller's workspace
struct WsLayout {
    size_t blocks, desc, parent, children, fbidx, leaves, leaf_of, orphans, orphan_idx, cfl_leaf,
        orphans_rest, orphan_rest_idx,
        restrict_list, prolong_list, prolong_mask, frame_list, frame_sel, reflux_slots, reflux_start, reflux_recs, sims,
        lvl_dx, dt, dt2, cfl_part,
        cond_part, tot_part, counters, fbuf, remap, newlist, shadow, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace mapk
