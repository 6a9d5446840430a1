// tile.hpp -- device-side addressing of the padded block tiles: linear index
// of a cell, the neighbour direction of a ghost cell, and where a padded cell
// of a block reads its value from (the ghost descriptors of Sec. 4.3 applied
// in place, so the update can read neighbour interiors without a copy).
#pragma once

#include <hip/hip_runtime.h>

#include "map_internal.hpp"

namespace mapk {

template <int NDIM>
constexpr int tile_cells() { return NDIM == 3 ? PD * PD * PD : PD * PD; }

// linear index of the cell (x, y, z) of a padded tile; coordinates are
// relative to the first interior cell (-NG .. NB+NG-1)
template <int NDIM>
__device__ __forceinline__ int lin(int x, int y, int z)
{
    if constexpr (NDIM == 3)
        return ((z + NG) * PD + (y + NG)) * PD + (x + NG);
    return (y + NG) * PD + (x + NG);
}

// direction index (dz+1)*9 + (dy+1)*3 + (dx+1) of the region holding (x, y, z)
template <int NDIM>
__device__ __forceinline__ int dir_index(int x, int y, int z)
{
    int dx = x < 0 ? -1 : (x >= NB ? 1 : 0);
    int dy = y < 0 ? -1 : (y >= NB ? 1 : 0);
    int dz = NDIM == 3 ? (z < 0 ? -1 : (z >= NB ? 1 : 0)) : 0;
    return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
}

// source index along one dimension: offset rule or CLAMP + fixed index
__device__ __forceinline__ int src_index(int g, int o) { return o >= CLAMP ? o - CLAMP : g + o; }

// Address of variable 0 of the value that padded cell (x, y, z) of block
// `slot` holds after a ghost fill: for a region whose descriptor names a
// same-level source, that source's interior cell (periodic wrap and outflow
// clamping are in the descriptor); otherwise the block's own cell (its
// interior, or a ghost prolongated from the parent).
// (element offset from the start of the state array)
template <int NDIM>
__device__ __forceinline__ size_t cell_src(const Desc *desc, int slot, int x, int y, int z)
{
    const Desc d = desc[(size_t)slot * NDIR + dir_index<NDIM>(x, y, z)];
    int s = slot;
    if (d.src >= 0) {
        s = d.src;
        x = src_index(x, d.o0);
        y = src_index(y, d.o1);
        if constexpr (NDIM == 3)
            z = src_index(z, d.o2);
    }
    return (size_t)s * NV * tile_cells<NDIM>() + lin<NDIM>(x, y, z);
}

}  // namespace mapk
