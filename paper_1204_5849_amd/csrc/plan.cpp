// plan.cpp -- host runtime: block-tree validation, Morton ordering and the
// tables the kernels read.  This is the single-GPU counterpart of the
// neighbour statistics of Sec. 4.2: everything a step needs to find
// its neighbours, parents, children and reflux partners is computed once here.
#include "keymap.hpp"
#include "plan.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

using namespace mapk;

uint64_t map_morton3(uint32_t x, uint32_t y, uint32_t z)
{
    auto spread = [](uint64_t v) {
        v &= 0x1fffff;
        v = (v | v << 32) & 0x1f00000000ffffULL;
        v = (v | v << 16) & 0x1f0000ff0000ffULL;
        v = (v | v << 8) & 0x100f00f00f00f00fULL;
        v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
        v = (v | v << 2) & 0x1249249249249249ULL;
        return v;
    };
    return spread(x) | spread(y) << 1 | spread(z) << 2;
}

namespace {

uint64_t pack(int sim, int level, int ix, int iy, int iz)
{
    return ((uint64_t)sim << 47) | ((uint64_t)level << 42) | ((uint64_t)ix << 28) |
           ((uint64_t)iy << 14) | (uint64_t)iz;
}

struct Tree {
    mapk::KeyMap slot;
    int find(int s, int l, int x, int y, int z) const { return slot.find(pack(s, l, x, y, z)); }
};

int blocks_at(const map_sim_desc &s, int d, int level) { return s.nbase[d] << (level - 1); }

}  // namespace

map_status map_plan_build(map_ctx *c, const map_params *p, int nsims, const map_sim_desc *sims,
                          int nblocks, const map_block_key *keys, std::string &err)
{
    if (!p || !sims || !keys || nsims <= 0 || nblocks <= 0) {
        err = "null pointer or empty list";
        return MAP_EINVAL;
    }
    if (p->ndim != 2 && p->ndim != 3) {
        err = "ndim must be 2 or 3";
        return MAP_EINVAL;
    }
    if (p->precision != MAP_FP64 && p->precision != MAP_FP32_MIXED) {
        err = "unknown precision";
        return MAP_EINVAL;
    }
    if (p->scheme != MAP_LF && p->scheme != MAP_MMC && p->scheme != MAP_WENO) {
        err = "unknown scheme";
        return MAP_EINVAL;
    }
    if (p->limiter < MAP_MINMOD || p->limiter > MAP_PAPER_PHI) {
        err = "unknown limiter";
        return MAP_EINVAL;
    }
    if (p->glm_mode != MAP_GLM_PAPER && p->glm_mode != MAP_GLM_FASTSPEED) {
        err = "unknown glm_mode";
        return MAP_EINVAL;
    }
    if (!(p->gamma > 1.0) || !(p->cfl > 0.0) || !(p->eta >= 0.0) ||
        (p->glm_mode == MAP_GLM_PAPER && !(p->glm_cd > 0.0 && p->glm_cd <= 1.0)) ||
        (p->glm_mode == MAP_GLM_FASTSPEED && !(p->glm_cr > 0.0))) {
        err = "gamma, cfl, eta, glm_cd or glm_cr out of range";
        return MAP_EINVAL;
    }
    if (p->riemann != MAP_RUSANOV && p->riemann != MAP_HLLC) {
        err = "unknown riemann solver";
        return MAP_EINVAL;
    }
    if (p->scheme == MAP_MMC && p->riemann != MAP_RUSANOV) {
        err = "MMC uses Lax-Friedrichs splitting, not a Riemann solver";
        return MAP_EINVAL;
    }
    if (p->cond_mode != MAP_COND_OFF && p->cond_mode != MAP_COND_ISO &&
        p->cond_mode != MAP_COND_FIELD) {
        err = "unknown cond_mode";
        return MAP_EINVAL;
    }
    if (p->cond_mode != MAP_COND_OFF) {
        const double h2 = 2.0 * p->kappa_exp;
        if (p->cond_max_sub < 1 || p->cond_max_sub > 64 || !(p->kappa0 >= 0.0) ||
            !(h2 >= 0.0 && h2 <= 10.0) || h2 != (double)(int)h2) {
            err = "conduction needs 1 <= cond_max_sub <= 64, kappa0 >= 0 and kappa_exp a "
                  "multiple of 1/2 in [0, 5]";
            return MAP_EINVAL;
        }
    }
    if (nsims >= (1 << 15)) {
        err = "too many simulations";
        return MAP_EINVAL;
    }
    const int nd = p->ndim;
    c->p = *p;
    c->nd = nd;
    c->tile = nd == 3 ? PD * PD * PD : PD * PD;
    c->word = p->precision == MAP_FP64 ? 8 : 4;
    c->sims.assign(sims, sims + nsims);
    for (int s = 0; s < nsims; s++) {
        for (int d = 0; d < 3; d++) {
            if (d < nd && (sims[s].nbase[d] <= 0 || !(sims[s].hi[d] > sims[s].lo[d]))) {
                err = "simulation " + std::to_string(s) + ": bad nbase or box";
                return MAP_EINVAL;
            }
            for (int side = 0; side < 2; side++)
                if (d < nd && sims[s].bc[d][side] != MAP_BC_PERIODIC &&
                    sims[s].bc[d][side] != MAP_BC_OUTFLOW) {
                    err = "unknown boundary kind";
                    return MAP_EINVAL;
                }
            if (d < nd && (sims[s].bc[d][0] == MAP_BC_PERIODIC) != (sims[s].bc[d][1] == MAP_BC_PERIODIC)) {
                err = "periodic boundaries must be periodic on both sides";
                return MAP_EINVAL;
            }
        }
        if (nd == 2 && sims[s].nbase[2] != 1) {
            err = "2-D simulations need nbase[2] == 1";
            return MAP_EINVAL;
        }
    }

    // ---- keys: range checks and duplicates
    Tree input;
    input.slot.reserve(nblocks);
    int lmax = 1;
    for (int i = 0; i < nblocks; i++) {
        const map_block_key &k = keys[i];
        if (k.sim < 0 || k.sim >= nsims || k.level < 1 || k.level > MAXL) {
            err = "key " + std::to_string(i) + ": bad sim or level";
            return MAP_ETREE;
        }
        const map_sim_desc &S = sims[k.sim];
        int co[3] = {k.ix, k.iy, k.iz};
        for (int d = 0; d < 3; d++) {
            int lim = d < nd ? blocks_at(S, d, k.level) : 1;
            if (co[d] < 0 || co[d] >= lim || lim >= (1 << 14)) {
                err = "key " + std::to_string(i) + ": coordinate out of range";
                return MAP_ETREE;
            }
        }
        uint64_t pk = pack(k.sim, k.level, k.ix, k.iy, k.iz);
        if (!input.slot.insert(pk, i)) {
            err = "key " + std::to_string(i) + ": duplicate block";
            return MAP_ETREE;
        }
        lmax = std::max(lmax, k.level);
    }
    c->lmax = lmax;

    // ---- parents, siblings, base completeness
    for (int i = 0; i < nblocks; i++) {
        const map_block_key &k = keys[i];
        if (k.level == 1)
            continue;
        if (input.find(k.sim, k.level - 1, k.ix >> 1, k.iy >> 1, k.iz >> 1) < 0) {
            err = "key " + std::to_string(i) + ": parent missing";
            return MAP_ETREE;
        }
        int nk = 1 << nd;
        for (int o = 0; o < nk; o++) {
            int sx = (k.ix & ~1) | (o & 1), sy = (k.iy & ~1) | ((o >> 1) & 1);
            int sz = nd == 3 ? ((k.iz & ~1) | ((o >> 2) & 1)) : 0;
            if (input.find(k.sim, k.level, sx, sy, sz) < 0) {
                err = "key " + std::to_string(i) + ": incomplete sibling set";
                return MAP_ETREE;
            }
        }
    }
    for (int s = 0; s < nsims; s++) {
        const map_sim_desc &S = sims[s];
        int nz = nd == 3 ? S.nbase[2] : 1;
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < S.nbase[1]; y++)
                for (int x = 0; x < S.nbase[0]; x++)
                    if (input.find(s, 1, x, y, z) < 0) {
                        err = "simulation " + std::to_string(s) + ": base level incomplete";
                        return MAP_ETREE;
                    }
    }

    // ---- 2:1 balance: every neighbour region of a block's parent exists at
    //      the parent's level (faces, edges and corners; periodic wrap)
    const int dzr = nd == 3 ? 1 : 0;
    for (int i = 0; i < nblocks; i++) {
        const map_block_key &k = keys[i];
        if (k.level <= 1)
            continue;
        const map_sim_desc &S = sims[k.sim];
        int pc[3] = {k.ix >> 1, k.iy >> 1, k.iz >> 1};
        for (int dz = -dzr; dz <= dzr; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int c3[3] = {pc[0] + dx, pc[1] + dy, pc[2] + dz};
                    bool skip = false;
                    for (int d = 0; d < nd; d++) {
                        int nbk = blocks_at(S, d, k.level - 1);
                        if (c3[d] < 0 || c3[d] >= nbk) {
                            if (S.bc[d][c3[d] < 0 ? 0 : 1] == MAP_BC_PERIODIC)
                                c3[d] = (c3[d] + nbk) % nbk;
                            else
                                skip = true;
                        }
                    }
                    if (!skip && input.find(k.sim, k.level - 1, c3[0], c3[1], c3[2]) < 0) {
                        err = "key " + std::to_string(i) + ": 2:1 balance violated";
                        return MAP_ETREE;
                    }
                }
    }

    // ---- Morton order: (sim, interleaved coordinates scaled to the finest
    //      level, level) puts every parent right before its children
    std::vector<int> order(nblocks);
    std::vector<uint64_t> mk(nblocks);
    for (int i = 0; i < nblocks; i++) {
        order[i] = i;
        int sh = lmax - keys[i].level;
        mk[i] = map_morton3((uint32_t)keys[i].ix << sh, (uint32_t)keys[i].iy << sh,
                            (uint32_t)keys[i].iz << sh);
    }
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        if (keys[a].sim != keys[b].sim) return keys[a].sim < keys[b].sim;
        if (mk[a] != mk[b]) return mk[a] < mk[b];
        return keys[a].level < keys[b].level;
    });
    const int n = nblocks;
    c->nslots = n;
    c->slot_of_key.assign(n, -1);
    c->key.resize(n);
    Tree tr;
    tr.slot.reserve(n);
    for (int s = 0; s < n; s++) {
        c->slot_of_key[order[s]] = s;
        c->key[s] = keys[order[s]];
        tr.slot.insert(pack(c->key[s].sim, c->key[s].level, c->key[s].ix, c->key[s].iy, c->key[s].iz), s);
    }

    // ---- parent / children / leaves
    c->parent.assign(n, -1);
    c->children.assign((size_t)n * 8, -1);
    c->blk.resize(n);
    for (int s = 0; s < n; s++) {
        const map_block_key &k = c->key[s];
        c->blk[s].sim = k.sim;
        c->blk[s].level = k.level;
        c->blk[s].cpos = (k.ix & 1) | ((k.iy & 1) << 1) | ((k.iz & 1) << 2);
        c->blk[s].leaf = 1;
        if (k.level > 1)
            c->parent[s] = tr.find(k.sim, k.level - 1, k.ix >> 1, k.iy >> 1, k.iz >> 1);
    }
    for (int s = 0; s < n; s++) {
        int ps = c->parent[s];
        if (ps >= 0) {
            c->blk[ps].leaf = 0;
            c->children[(size_t)ps * 8 + c->blk[s].cpos] = s;
        }
    }
    c->leaves.clear();
    c->leaf_of.assign(n, -1);
    c->orphans.clear();
    c->orphan_idx.clear();
    for (int s = 0; s < n; s++)
        if (c->blk[s].leaf) {
            c->leaf_of[s] = (int32_t)c->leaves.size();
            if (c->parent[s] < 0) {
                c->orphans.push_back(s);
                c->orphan_idx.push_back((int32_t)c->leaves.size());
            }
            c->leaves.push_back(s);
        }
    c->nleaves = (int)c->leaves.size();

    // ---- per-simulation records: leaf ranges (leaves are grouped by sim),
    //      cell widths per level, smallest leaf width
    c->simrec.assign(nsims, SimRec{0.0, 0, 0});
    c->lvl_dx.assign((size_t)nsims * (MAXL + 1) * 3, 1.0);
    for (int s = 0; s < nsims; s++)
        for (int l = 1; l <= MAXL; l++)
            for (int d = 0; d < nd; d++)
                c->lvl_dx[((size_t)s * (MAXL + 1) + l) * 3 + d] =
                    (sims[s].hi[d] - sims[s].lo[d]) / (double)(blocks_at(sims[s], d, l) * NB);
    {
        int li = 0;
        for (int s = 0; s < nsims; s++) {
            c->simrec[s].leaf_lo = li;
            double dxmin = 0.0;
            bool first = true;
            while (li < c->nleaves && c->blk[c->leaves[li]].sim == s) {
                int l = c->blk[c->leaves[li]].level;
                for (int d = 0; d < nd; d++) {
                    double v = c->lvl_dx[((size_t)s * (MAXL + 1) + l) * 3 + d];
                    if (first || v < dxmin) {
                        dxmin = v;
                        first = false;
                    }
                }
                li++;
            }
            c->simrec[s].leaf_hi = li;
            c->simrec[s].dxmin = dxmin;
        }
    }

    // ---- ghost descriptors: per direction, the same-level block that holds
    //      the source cells after periodic wrap or outflow clamping, or -1
    //      when the region is covered only by a coarser block (prolongate)
    c->desc.assign((size_t)n * NDIR, Desc{-2, 0, 0, 0});
    for (int s = 0; s < n; s++) {
        const map_block_key &k = c->key[s];
        const map_sim_desc &S = sims[k.sim];
        int kc[3] = {k.ix, k.iy, k.iz};
        for (int dz = -dzr; dz <= dzr; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    if (!dx && !dy && !dz)
                        continue;
                    int dir[3] = {dx, dy, dz};
                    int src[3], off[3] = {0, 0, 0};
                    for (int d = 0; d < 3; d++) {
                        src[d] = kc[d];
                        if (d >= nd || dir[d] == 0)
                            continue;
                        int nbk = blocks_at(S, d, k.level);
                        int nc = kc[d] + dir[d];
                        if (nc >= 0 && nc < nbk) {
                            src[d] = nc;
                            off[d] = -dir[d] * NB;
                        } else if (S.bc[d][dir[d] < 0 ? 0 : 1] == MAP_BC_PERIODIC) {
                            src[d] = (nc + nbk) % nbk;
                            off[d] = -dir[d] * NB;
                        } else {
                            src[d] = kc[d];  // zero-gradient: the edge cell of this block
                            off[d] = CLAMP + (dir[d] < 0 ? 0 : NB - 1);
                        }
                    }
                    int ss = tr.find(k.sim, k.level, src[0], src[1], src[2]);
                    int di = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                    c->desc[(size_t)s * NDIR + di] = Desc{ss >= 0 ? ss : -1, off[0], off[1], off[2]};
                }
    }

    // ---- restriction lists (parents by level) and prolongation lists
    c->restrict_list.clear();
    c->restrict_off.assign(lmax + 2, 0);
    for (int l = 1; l <= lmax; l++) {
        c->restrict_off[l] = (int)c->restrict_list.size();
        for (int s = 0; s < n; s++)
            if (c->blk[s].level == l && !c->blk[s].leaf)
                c->restrict_list.push_back(s);
    }
    c->restrict_off[lmax + 1] = (int)c->restrict_list.size();
    c->prolong_list.clear();
    c->prolong_mask.clear();
    c->prolong_off.assign(lmax + 2, 0);
    for (int l = 1; l <= lmax; l++) {
        c->prolong_off[l] = (int)c->prolong_list.size();
        for (int s = 0; s < n; s++) {
            if (c->blk[s].level != l)
                continue;
            uint32_t m = 0;
            for (int di = 0; di < NDIR; di++)
                if (di != 13 && c->desc[(size_t)s * NDIR + di].src == -1)
                    m |= 1u << di;
            if (m) {
                c->prolong_list.push_back(s);
                c->prolong_mask.push_back(m);
            }
        }
    }
    c->prolong_off[lmax + 1] = (int)c->prolong_list.size();
    // parents whose padded tiles the prolongation reads: the update reads
    // same-level neighbour interiors in place, so within a cycle only these
    // ghost frames are filled by copies
    {
        std::vector<char> mark(n, 0);
        for (int s : c->prolong_list)
            if (c->parent[s] >= 0)
                mark[c->parent[s]] = 1;
        c->frame_list.clear();
        for (int s = 0; s < n; s++)
            if (mark[s])
                c->frame_list.push_back(s);
    }
    // the ghost cells of those parent tiles that the stencil of the
    // minmod-limited prolongation reads, as the directions they lie in and
    // their bounding box: fine ghost cell f (per dimension, counted from the
    // parent's lowest interior cell) takes the parent cell floor(f / 2) and
    // its two neighbours along each dimension in turn
    {
        auto fdiv2 = [](int v) { return v >= 0 ? v / 2 : -((1 - v) / 2); };
        // bit b of the result: dimension range [lo, hi] meets side b - 1
        // (below the interior, inside it, above it)
        auto sides = [](int lo, int hi) {
            return (lo < 0 ? 1u : 0u) | (lo < NB && hi >= 0 ? 2u : 0u) | (hi >= NB ? 4u : 0u);
        };
        std::vector<uint32_t> mask(n, 0);
        std::vector<std::array<int, 6>> box(n, {NB, NB, NB, -1, -1, -1});
        for (int s : c->prolong_list) {
            const int p = c->parent[s];
            if (p < 0)
                continue;
            const int cpos = c->blk[s].cpos;
            for (int di = 0; di < NDIR; di++) {
                if (di == 13 || c->desc[(size_t)s * NDIR + di].src != -1)
                    continue;
                const int dir[3] = {di % 3 - 1, (di / 3) % 3 - 1, di / 9 - 1};
                int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
                for (int d = 0; d < nd; d++) {
                    const int base = ((cpos >> d) & 1) * NB;
                    const int a = dir[d] < 0 ? -NG : (dir[d] > 0 ? NB : 0);
                    const int b = dir[d] < 0 ? -1 : (dir[d] > 0 ? NB + NG - 1 : NB - 1);
                    lo[d] = fdiv2(base + a);
                    hi[d] = fdiv2(base + b);
                }
                for (int e = -1; e < nd; e++) {  // the centre cells, then each dimension's pair
                    uint32_t sd[3];
                    for (int d = 0; d < 3; d++) {
                        sd[d] = d < nd ? sides(lo[d] - (d == e), hi[d] + (d == e)) : 2u;
                        box[p][d] = std::min(box[p][d], lo[d] - (d == e));
                        box[p][3 + d] = std::max(box[p][3 + d], hi[d] + (d == e));
                    }
                    for (int z = 0; z < 3; z++)
                        for (int y = 0; y < 3; y++)
                            for (int x = 0; x < 3; x++)
                                if ((sd[0] >> x & 1) && (sd[1] >> y & 1) && (sd[2] >> z & 1) &&
                                    z * 9 + y * 3 + x != 13)
                                    mask[p] |= 1u << (z * 9 + y * 3 + x);
                }
            }
        }
        c->frame_sel.clear();
        for (int s : c->frame_list) {
            FrameSel f{};
            f.dirs = mask[s];
            for (int d = 0; d < 3; d++) {
                f.lo[d] = box[s][d];
                f.hi[d] = box[s][3 + d];
            }
            c->frame_sel.push_back(f);
        }
    }

    // ---- reflux: coarse leaf faces whose same-level neighbour has children
    c->fbidx.assign((size_t)n * 6, -1);
    c->nfb = 0;
    auto fb_of = [&](int s, int face) {
        int &v = c->fbidx[(size_t)s * 6 + face];
        if (v < 0)
            v = c->nfb++;
        return v;
    };
    c->reflux_slots.clear();
    c->reflux_start.clear();
    c->reflux_recs.clear();
    for (int s = 0; s < n; s++) {
        if (!c->blk[s].leaf)
            continue;
        const map_block_key &k = c->key[s];
        const map_sim_desc &S = sims[k.sim];
        int kc[3] = {k.ix, k.iy, k.iz};
        bool started = false;
        for (int d = 0; d < nd; d++) {
            int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            for (int side = 0; side < 2; side++) {
                int nbk = blocks_at(S, d, k.level);
                int nc[3] = {kc[0], kc[1], kc[2]};
                nc[d] += side ? 1 : -1;
                if (nc[d] < 0 || nc[d] >= nbk) {
                    if (S.bc[d][side] != MAP_BC_PERIODIC)
                        continue;
                    nc[d] = (nc[d] + nbk) % nbk;
                }
                int nb = tr.find(k.sim, k.level, nc[0], nc[1], nc[2]);
                if (nb < 0 || c->blk[nb].leaf)
                    continue;
                if (!started) {
                    c->reflux_slots.push_back(s);
                    c->reflux_start.push_back((int)c->reflux_recs.size());
                    started = true;
                }
                RefluxRec r{};
                r.dim = d;
                r.side = side;
                r.fb_coarse = fb_of(s, 2 * d + side);
                int nf = nd == 3 ? 4 : 2;
                for (int o = 0; o < 4; o++)
                    r.fb_fine[o] = -1;
                for (int o = 0; o < nf; o++) {
                    int fc[3];
                    fc[d] = 2 * nc[d] + (side ? 0 : 1);
                    fc[t1] = 2 * kc[t1] + (o & 1);
                    fc[t2] = nd == 3 ? 2 * kc[t2] + ((o >> 1) & 1) : 0;
                    int fs = tr.find(k.sim, k.level + 1, fc[0], fc[1], fc[2]);
                    if (fs < 0 || !c->blk[fs].leaf) {
                        err = "reflux partner missing (tree not 2:1 balanced)";
                        return MAP_ETREE;
                    }
                    r.fb_fine[o] = fb_of(fs, 2 * d + (1 - side));
                }
                c->reflux_recs.push_back(r);
            }
        }
    }
    c->reflux_start.push_back((int)c->reflux_recs.size());

    // ---- leaves without parent whose next-cycle CFL maximum the 2-D LF
    //      update forms as it writes them (reflux would change them after
    //      the update, so leaves with reflux faces stay with the CFL pass)
    c->cfl_leaf.assign(n, -1);
    c->orphans_rest.clear();
    c->orphan_rest_idx.clear();
    {
        std::vector<char> refl(n, 0);
        for (int s : c->reflux_slots)
            refl[s] = 1;
        const bool can = nd == 2 && p->scheme == MAP_LF;
        for (size_t i = 0; i < c->orphans.size(); i++) {
            const int s = c->orphans[i];
            if (can && !refl[s]) {
                c->cfl_leaf[s] = c->orphan_idx[i];
            } else {
                c->orphans_rest.push_back(s);
                c->orphan_rest_idx.push_back(c->orphan_idx[i]);
            }
        }
    }
    map_plan_layout(c);
    return MAP_OK;
}

void map_plan_layout(map_ctx *c)
{
    WsLayout &L = c->ws;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t n = c->nslots, ns = c->sims.size();
    L.blocks = take(n * sizeof(BlockRec));
    L.desc = take(n * NDIR * sizeof(Desc));
    L.parent = take(n * sizeof(int32_t));
    L.children = take(n * 8 * sizeof(int32_t));
    L.fbidx = take(n * 6 * sizeof(int32_t));
    L.leaves = take((size_t)c->nleaves * sizeof(int32_t));
    L.leaf_of = take(n * sizeof(int32_t));
    L.orphans = take(c->orphans.size() * sizeof(int32_t));
    L.orphan_idx = take(c->orphan_idx.size() * sizeof(int32_t));
    L.cfl_leaf = take(n * sizeof(int32_t));
    L.orphans_rest = take(c->orphans_rest.size() * sizeof(int32_t));
    L.orphan_rest_idx = take(c->orphan_rest_idx.size() * sizeof(int32_t));
    L.restrict_list = take(c->restrict_list.size() * sizeof(int32_t));
    L.prolong_list = take(c->prolong_list.size() * sizeof(int32_t));
    L.prolong_mask = take(c->prolong_mask.size() * sizeof(uint32_t));
    L.frame_list = take(c->frame_list.size() * sizeof(int32_t));
    L.frame_sel = take(c->frame_sel.size() * sizeof(FrameSel));
    L.reflux_slots = take(c->reflux_slots.size() * sizeof(int32_t));
    L.reflux_start = take(c->reflux_start.size() * sizeof(int32_t));
    L.reflux_recs = take(c->reflux_recs.size() * sizeof(RefluxRec));
    L.sims = take(ns * sizeof(SimRec));
    L.lvl_dx = take(c->lvl_dx.size() * sizeof(double));
    L.dt = take(ns * sizeof(map_dt));
    L.dt2 = take(ns * sizeof(map_dt));
    L.cfl_part = take((size_t)c->nleaves * sizeof(double));
    L.cond_part = take((size_t)c->nleaves * sizeof(double));
    L.tot_part = take((size_t)c->nleaves * NV * sizeof(double));
    L.counters = take(4 * sizeof(unsigned long long));
    L.fbuf = take((size_t)c->nfb * NV * c->face_cells() * c->word);
    L.remap = take(n * sizeof(int32_t));
    L.newlist = take(n * sizeof(int32_t));
    L.shadow = take(n * NV * (size_t)c->tile * c->word);
    L.total = o;
}
