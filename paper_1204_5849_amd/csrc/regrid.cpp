// regrid.cpp -- the host tree edit of one regrid (paper Sec. 4.5): refine
// flagged leaves, destroy the children of smooth blocks, close the result
// under 2:1 balance.  Host only; the estimates come from map_estimate.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "keymap.hpp"
#include "plan.hpp"

using namespace mapk;

namespace {

// (sim, level, ix, iy, iz) packed into 62 bits: coordinates are < 2^14 and
// levels < 32 (both checked when the tree was planned)
inline uint64_t pack(int sim, int lv, int x, int y, int z)
{
    return ((uint64_t)sim << 47) | ((uint64_t)lv << 42) | ((uint64_t)x << 28) |
           ((uint64_t)y << 14) | (uint64_t)z;
}
inline map_block_key unpack(uint64_t k)
{
    map_block_key b;
    b.sim = (int)(k >> 47);
    b.level = (int)((k >> 42) & 31);
    b.ix = (int)((k >> 28) & 16383);
    b.iy = (int)((k >> 14) & 16383);
    b.iz = (int)(k & 16383);
    return b;
}
inline uint64_t parent_of(uint64_t k)
{
    map_block_key b = unpack(k);
    return pack(b.sim, b.level - 1, b.ix >> 1, b.iy >> 1, b.iz >> 1);
}

}  // namespace

extern map_status regrid_fail(map_status st, const std::string &msg);

extern "C" map_status map_regrid(const map_ctx *c, const double *err, const map_regrid_params *rp,
                                 map_block_key *keys_out, int capacity, int *nout)
{
    if (!c || !err || !rp || !nout || capacity < 0 || (capacity > 0 && !keys_out))
        return regrid_fail(MAP_EINVAL, "null argument or negative capacity");
    if (rp->max_level < 1 || rp->max_level > MAXL)
        return regrid_fail(MAP_EINVAL, "max_level out of range");
    const int n = c->nslots, nd = c->nd;
    const int nkids = 1 << nd;
    KeyMap slot_of(n);
    for (int s = 0; s < n; s++) {
        const map_block_key &k = c->key[s];
        slot_of.insert(pack(k.sim, k.level, k.ix, k.iy, k.iz), s);
    }
    auto kids_of = [&](int s) {
        const map_block_key &k = c->key[s];
        std::vector<uint64_t> out;
        for (int o = 0; o < nkids; o++)
            out.push_back(pack(k.sim, k.level + 1, 2 * k.ix + (o & 1), 2 * k.iy + ((o >> 1) & 1),
                               nd == 3 ? 2 * k.iz + ((o >> 2) & 1) : 0));
        return out;
    };

    // first decisions
    std::vector<char> refine(n, 0), coarsen(n, 0);
    for (int s = 0; s < n; s++)
        if (c->blk[s].leaf && err[s] > rp->tau_refine && c->key[s].level < rp->max_level)
            refine[s] = 1;
    for (int s = 0; s < n; s++) {
        if (c->blk[s].leaf || !(err[s] < rp->tau_coarsen))
            continue;
        bool ok = true;
        for (int o = 0; o < nkids; o++) {
            const int ch = c->children[(size_t)s * 8 + o];
            ok = ok && ch >= 0 && c->blk[ch].leaf && !refine[ch];
        }
        coarsen[s] = ok;
    }

    // closure: a new leaf must not touch a leaf two or more levels coarser
    KeyMap leaves(n * nkids);
    for (;;) {
        leaves.clear();
        for (int s = 0; s < n; s++) {
            const map_block_key &k = c->key[s];
            if (c->blk[s].leaf) {
                const int p = c->parent[s];
                if (p >= 0 && coarsen[p])
                    continue;
                if (refine[s]) {
                    for (uint64_t ch : kids_of(s))
                        leaves.insert(ch, 0);
                } else {
                    leaves.insert(pack(k.sim, k.level, k.ix, k.iy, k.iz), 0);
                }
            } else if (coarsen[s]) {
                leaves.insert(pack(k.sim, k.level, k.ix, k.iy, k.iz), 0);
            }
        }
        std::vector<uint64_t> order(leaves.keys());
        std::sort(order.begin(), order.end());
        bool changed = false;
        for (uint64_t a : order) {
            const map_block_key ka = unpack(a);
            const map_sim_desc &S = c->sims[ka.sim];
            const int ac[3] = {ka.ix, ka.iy, ka.iz};
            const int dzr = nd == 3 ? 1 : 0;
            for (int dz = -dzr; dz <= dzr; dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        if (!dx && !dy && !dz)
                            continue;
                        const int dd[3] = {dx, dy, dz};
                        int nc[3] = {0, 0, 0};
                        bool inside = true;
                        for (int d = 0; d < nd && inside; d++) {
                            const int nb = S.nbase[d] << (ka.level - 1);
                            int v = ac[d] + dd[d];
                            if (v < 0 || v >= nb) {
                                if (S.bc[d][v < 0 ? 0 : 1] != MAP_BC_PERIODIC)
                                    inside = false;
                                v = (v + nb) % nb;
                            }
                            nc[d] = v;
                        }
                        if (!inside)
                            continue;
                        // the new leaf covering the neighbour region, if coarser
                        for (int bl = ka.level - 1; bl >= 1; bl--) {
                            const int sh = ka.level - bl;
                            const uint64_t b = pack(ka.sim, bl, nc[0] >> sh, nc[1] >> sh, nc[2] >> sh);
                            if (!leaves.contains(b))
                                continue;
                            if (bl <= ka.level - 2) {
                                const int sb = slot_of.find(b);
                                if (sb < 0)
                                    return regrid_fail(MAP_ETREE, "input tree is not 2:1 balanced");
                                if (coarsen[sb]) {
                                    coarsen[sb] = 0;
                                } else {
                                    refine[sb] = 1;
                                    const int pb = c->parent[sb];
                                    if (pb >= 0)
                                        coarsen[pb] = 0;
                                }
                                changed = true;
                            }
                            break;
                        }
                    }
        }
        if (!changed)
            break;
    }

    // the new tree: the new leaves and all their ancestors
    KeyMap all(2 * leaves.size());
    for (uint64_t k : leaves.keys())
        all.insert(k, 0);
    for (uint64_t k : leaves.keys())
        for (uint64_t a = k; unpack(a).level > 1;) {
            a = parent_of(a);
            if (!all.insert(a, 0))
                break;
        }
    std::vector<map_block_key> out;
    out.reserve(all.size());
    for (uint64_t k : all.keys())
        out.push_back(unpack(k));
    std::sort(out.begin(), out.end(), [](const map_block_key &x, const map_block_key &y) {
        if (x.sim != y.sim)
            return x.sim < y.sim;
        if (x.level != y.level)
            return x.level < y.level;
        if (x.ix != y.ix)
            return x.ix < y.ix;
        if (x.iy != y.iy)
            return x.iy < y.iy;
        return x.iz < y.iz;
    });
    *nout = (int)out.size();
    if ((int)out.size() > capacity)
        return regrid_fail(MAP_ENOMEM, "keys_out holds " + std::to_string(capacity) + " keys, need " +
                                           std::to_string(out.size()));
    std::memcpy(keys_out, out.data(), out.size() * sizeof(map_block_key));
    return MAP_OK;
}

// The interval to the next regrid (Sec. 4.5): the time the fastest wave
// needs to cross the 2 n_g cells of the buffer zone that the estimate
// covers, at the simulation's finest leaf cell width.
extern "C" map_status map_regrid_interval(const map_ctx *c, const map_dt *dt_host, double c_r,
                                          double *dtr_host, int *steps_host)
{
    if (!c || !dt_host || !dtr_host || !steps_host)
        return regrid_fail(MAP_EINVAL, "null argument");
    if (!(c_r > 0.0))
        return regrid_fail(MAP_EINVAL, "c_r must be positive");
    for (size_t s = 0; s < c->simrec.size(); s++) {
        const double dt = dt_host[s].dt, alpha = dt_host[s].alpha;
        if (!(dt > 0.0) || !(alpha >= 0.0))
            return regrid_fail(MAP_EINVAL, "dt record " + std::to_string(s) + " has no positive dt");
        const double dtr = alpha > 0.0 ? c_r * 2.0 * NG * c->simrec[s].dxmin / alpha : HUGE_VAL;
        dtr_host[s] = dtr;
        const double n = std::floor(dtr / dt);
        steps_host[s] = n < 1.0 ? 1 : (n > 1e9 ? 1000000000 : (int)n);
    }
    return MAP_OK;
}
