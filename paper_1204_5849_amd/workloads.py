"""Seeded synthetic workloads: block lists and primitive initial data.

This module is the only code shared by the HIP path and the FP64 oracle.  It
holds none of the method's arithmetic: it lays out block keys (geometric
refinement only), evaluates analytic initial conditions in *primitive*
variables (rho, v_x, v_y, v_z, B_x, B_y, B_z, p, psi) at cell centres in FP64
(point values are taken as cell averages, Sec. 3 of the paper), and draws
seeded noise from a counter-based splitmix64 (Steele, Lea & Flood 2014) keyed
on (seed, sim, level, global cell index, component), so both sides receive
identical inputs whatever the decomposition.  Conversion to conserved
variables, restriction and ghost fill are the method's and happen on each
side separately.

Problems (sizes as stated by each builder):
  orszag_tang     2-D Orszag-Tang vortex on a uniform block grid
  ot_amr          the same vortex on a given static AMR block list
  blast3d         3-D MHD blast wave, base 128^3, refined sphere
  harris3d        3-D Harris current sheet, 4 levels refined towards y=0
  kh_ensemble     many 2-D Kelvin-Helmholtz runs of uneven sizes
  alfven2d, advection1d, advection2d   smooth problems for convergence tests
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Sequence

import numpy as np

NVAR = 9
RHO, VX, VY, VZ, BX, BY, BZ, PR, PSI = range(9)


@dataclass
class SimDesc:
    lo: Sequence[float]
    hi: Sequence[float]
    nbase: Sequence[int]
    bc: Sequence[Sequence[str]]  # per dim (low, high): "periodic" | "outflow"


@dataclass
class Workload:
    name: str
    ndim: int
    sims: List[SimDesc]
    keys: np.ndarray                # [nb, 5] int32: sim, level, ix, iy, iz
    ic: Callable                    # ic(wl, sim, level, x, y, z, gidx) -> [9, ...] primitives
    n: int = 16
    scheme: str = "lf"
    limiter: str = "minmod"
    riemann: str = "rusanov"        # face flux of LF and WENO: "rusanov" or "hllc"
    cond: str = "off"               # thermal conduction: "off", "iso", "field"
    cond_max_sub: int = 8           # conduction sub-steps per step at most
    kappa0: float = 0.0             # kappa = kappa0 T^kappa_exp
    kappa_exp: float = 2.5
    glm_mode: str = "paper"
    eglm_sources: bool = True
    gamma: float = 5.0 / 3.0
    cfl: float = 0.4
    cd: float = 0.18
    cr: float = 0.18
    eta: float = 0.0
    precision: str = "fp64"
    steps: int = 100
    seed: int = 1204
    extra: dict = field(default_factory=dict)

    # ------------------------------------------------------------ geometry
    def cells_at_level(self, sim: int, d: int, level: int) -> int:
        return self.sims[sim].nbase[d] * self.n << (level - 1)

    def dx(self, sim: int, level: int):
        s = self.sims[sim]
        return [(s.hi[d] - s.lo[d]) / self.cells_at_level(sim, d, level) if d < self.ndim else 1.0
                for d in range(3)]

    def leaf_mask(self) -> np.ndarray:
        return leaf_mask(self.keys)

    def n_leaf_cells(self) -> int:
        return int(self.leaf_mask().sum()) * self.n ** self.ndim

    # ------------------------------------------------------------ initial data
    def primitive_blocks(self, blocks) -> np.ndarray:
        """Primitive interior values [len(blocks), 9, nz, ny, nx] (nz = 1 in 2-D),
        evaluated group by group (same sim and level) with array broadcasting."""
        blocks = np.asarray(blocks, dtype=np.int64)
        n = self.n
        nz = n if self.ndim == 3 else 1
        out = np.empty((len(blocks), NVAR, nz, n, n))
        if len(blocks) == 0:
            return out
        kb = self.keys[blocks]
        groups = {}
        for i, (sim, lv) in enumerate(zip(kb[:, 0].tolist(), kb[:, 1].tolist())):
            groups.setdefault((sim, lv), []).append(i)
        ar = np.arange(n)
        for (sim, lv), rows in groups.items():
            rows = np.asarray(rows)
            k = kb[rows]
            s = self.sims[sim]
            dx = self.dx(sim, lv)
            gx = (k[:, 2, None] * n + ar)[:, None, None, :]
            gy = (k[:, 3, None] * n + ar)[:, None, :, None]
            if self.ndim == 3:
                gz = (k[:, 4, None] * n + ar)[:, :, None, None]
                Z = s.lo[2] + (gz + 0.5) * dx[2]
            else:
                gz = np.zeros((len(rows), 1, 1, 1), dtype=np.int64)
                Z = np.zeros((len(rows), 1, 1, 1))
            X = s.lo[0] + (gx + 0.5) * dx[0]
            Y = s.lo[1] + (gy + 0.5) * dx[1]
            shape = (len(rows), nz, n, n)
            nx_l = np.uint64(self.cells_at_level(sim, 0, lv))
            ny_l = np.uint64(self.cells_at_level(sim, 1, lv))
            gidx = (gz.astype(np.uint64) * ny_l + gy.astype(np.uint64)) * nx_l + gx.astype(np.uint64)
            gidx = np.broadcast_to(gidx, shape)
            w = self.ic(self, sim, lv, np.broadcast_to(X, shape), np.broadcast_to(Y, shape),
                        np.broadcast_to(Z, shape), gidx)
            for c, val in enumerate(w):
                out[rows, c] = np.broadcast_to(np.asarray(val, dtype=np.float64), shape)
        return out


# ---------------------------------------------------------------- block lists
def leaf_mask(keys: np.ndarray) -> np.ndarray:
    keys = np.asarray(keys)
    parents = set()
    for s, lv, ix, iy, iz in keys:
        if lv > 1:
            parents.add((int(s), int(lv) - 1, int(ix) >> 1, int(iy) >> 1, int(iz) >> 1))
    return np.array([(int(s), int(lv), int(ix), int(iy), int(iz)) not in parents
                     for s, lv, ix, iy, iz in keys], dtype=bool)


def base_keys(sim: int, nbase, ndim: int) -> np.ndarray:
    nz = nbase[2] if ndim == 3 else 1
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(nbase[1]), np.arange(nbase[0]),
                             indexing="ij")
    k = np.stack([np.full(ix.size, sim), np.ones(ix.size, dtype=int), ix.ravel(), iy.ravel(),
                  iz.ravel()], axis=1)
    return k.astype(np.int32)


def children_of(keys: np.ndarray, ndim: int) -> np.ndarray:
    out = []
    for s, lv, ix, iy, iz in keys:
        for o in range(1 << ndim):
            cz = (o >> 2) & 1 if ndim == 3 else 0
            out.append((s, lv + 1, 2 * ix + (o & 1), 2 * iy + ((o >> 1) & 1), 2 * iz + cz))
    return np.array(out, dtype=np.int32).reshape(-1, 5)


def block_bounds(wl_n: int, sim: SimDesc, level: int, key, ndim: int):
    lo, hi = [], []
    for d in range(ndim):
        w = (sim.hi[d] - sim.lo[d]) / (sim.nbase[d] << (level - 1))
        i = key[2 + d]
        lo.append(sim.lo[d] + i * w)
        hi.append(sim.lo[d] + (i + 1) * w)
    return lo, hi


def refine_geometric(sims, ndim, levels, predicate) -> np.ndarray:
    """Base blocks of every sim, then at each level refine the leaves for which
    predicate(sim_index, level, lo, hi) is true."""
    keys = [base_keys(i, s.nbase, ndim) for i, s in enumerate(sims)]
    allk = np.concatenate(keys)
    current = allk
    for lv in range(1, levels):
        sel = np.array([predicate(int(k[0]), lv, *block_bounds(0, sims[k[0]], lv, k, ndim))
                        for k in current], dtype=bool)
        kids = children_of(current[sel], ndim)
        if len(kids) == 0:
            break
        allk = np.concatenate([allk, kids])
        current = kids
    return allk


# ---------------------------------------------------------------- seeded noise
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    """splitmix64 finaliser applied to uint64 counters (wrapping arithmetic)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def counter_uniform(seed, sim, level, gidx, comp):
    """Uniform [-1, 1) from the counter (seed, sim, level, gidx, comp)."""
    h = splitmix64(np.uint64(seed))
    h = splitmix64(h ^ np.uint64(sim))
    h = splitmix64(h ^ np.uint64(level))
    h = splitmix64(h ^ np.asarray(gidx, dtype=np.uint64))
    h = splitmix64(h ^ np.uint64(comp))
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


# ---------------------------------------------------------------- problems
def _ot_ic(wl, sim, lv, x, y, z, gidx):
    tp = 2.0 * math.pi
    s4 = 1.0 / math.sqrt(4.0 * math.pi)
    return [25.0 / (36.0 * math.pi), -np.sin(tp * y), np.sin(tp * x), 0.0,
            -np.sin(tp * y) * s4, np.sin(2.0 * tp * x) * s4, 0.0, 5.0 / (12.0 * math.pi), 0.0]


def _unit_square(nb):
    return SimDesc(lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), nbase=(nb, nb, 1),
                   bc=(("periodic", "periodic"),) * 3)


def orszag_tang(nbase: int = 8, steps: int = 100, precision="fp64", scheme="lf",
                limiter="minmod") -> Workload:
    """2-D Orszag-Tang, periodic unit square, (16 nbase)^2 cells, uniform."""
    sims = [_unit_square(nbase)]
    return Workload(name=f"orszag_tang_{16 * nbase}", ndim=2, sims=sims,
                    keys=base_keys(0, sims[0].nbase, 2), ic=_ot_ic, steps=steps,
                    precision=precision, scheme=scheme, limiter=limiter)


def ot_amr(keys: np.ndarray, nbase: int = 16, steps: int = 500, precision="fp64") -> Workload:
    """2-D Orszag-Tang on a static AMR block list (base (16 nbase)^2),
    modified MacCormack + van Leer."""
    sims = [_unit_square(nbase)]
    return Workload(name="orszag_tang_amr", ndim=2, sims=sims,
                    keys=np.asarray(keys, dtype=np.int32), ic=_ot_ic, steps=steps,
                    precision=precision, scheme="mmc", limiter="vanleer")


def _blast_ic(wl, sim, lv, x, y, z, gidx):
    r2 = x * x + y * y + z * z
    p = np.where(r2 < 0.01, 100.0, 0.1)
    s = 1.0 / math.sqrt(2.0)
    return [1.0, 0.0, 0.0, 0.0, s, s, 0.0, p, 0.0]


def blast3d(nbase: int = 8, levels: int = 2, r_refine: float = 0.3, steps: int = 100,
            precision="fp32") -> Workload:
    """3-D blast on [-0.5,0.5]^3 periodic, base (16 nbase)^3; blocks meeting
    r <= r_refine are refined at each level."""
    sims = [SimDesc(lo=(-0.5, -0.5, -0.5), hi=(0.5, 0.5, 0.5), nbase=(nbase,) * 3,
                    bc=(("periodic", "periodic"),) * 3)]

    def pred(si, lv, lo, hi):
        d2 = 0.0
        for a, b in zip(lo, hi):
            c = min(max(0.0, a), b)
            d2 += c * c
        return d2 <= r_refine * r_refine

    keys = refine_geometric(sims, 3, levels, pred)
    return Workload(name=f"blast3d_{16 * nbase}_L{levels}", ndim=3, sims=sims, keys=keys,
                    ic=_blast_ic, steps=steps, precision=precision, glm_mode="fastspeed")


def _harris_ic(wl, sim, lv, x, y, z, gidx):
    w = 0.5
    sech2 = 1.0 / np.cosh(y / w) ** 2
    amp = wl.extra.get("noise", 1e-3)
    vx = amp * counter_uniform(wl.seed, sim, lv, gidx, 0)
    vy = amp * counter_uniform(wl.seed, sim, lv, gidx, 1)
    vz = amp * counter_uniform(wl.seed, sim, lv, gidx, 2)
    return [1.0 + sech2, vx, vy, vz, np.tanh(y / w), 0.0, 0.0, 0.1 + 0.5 * sech2, 0.0]


def harris3d(nbase: int = 8, levels: int = 4, steps: int = 100, precision="fp32",
             half_width: float = 2.0) -> Workload:
    """3-D Harris sheet on [-2,2]^3, periodic x,z, outflow y, eta = 1e-3, base
    (16 nbase)^3; a block at level l is refined where its y-range meets
    |y| < 0.5 / 2^(l-1)."""
    L = half_width
    sims = [SimDesc(lo=(-L, -L, -L), hi=(L, L, L), nbase=(nbase,) * 3,
                    bc=(("periodic", "periodic"), ("outflow", "outflow"),
                        ("periodic", "periodic")))]

    def pred(si, lv, lo, hi):
        lim = 0.5 / (1 << (lv - 1))
        return lo[1] < lim and hi[1] > -lim

    keys = refine_geometric(sims, 3, levels, pred)
    return Workload(name=f"harris3d_{16 * nbase}_L{levels}", ndim=3, sims=sims, keys=keys,
                    ic=_harris_ic, steps=steps, precision=precision, glm_mode="fastspeed",
                    eta=1e-3)


def _kh_ic(wl, sim, lv, x, y, z, gidx):
    m, phi = wl.extra["modes"][sim]
    return [1.0, 0.5 * np.tanh(y / 0.05), 0.01 * np.sin(2.0 * math.pi * m * x + phi), 0.0,
            0.1, 0.0, 0.0, 1.0, 0.0]


def kh_sizes(nsims: int, seed: int, kmin: int = 4, kmax: int = 32):
    """Blocks per side k in {kmin..kmax}, mode m in {1..4} and phase in [0, 2pi)
    for each run, drawn from splitmix64 counters."""
    ks, modes = [], []
    for i in range(nsims):
        h = int(splitmix64(splitmix64(np.uint64(seed)) ^ np.uint64(i)))
        ks.append(kmin + h % (kmax - kmin + 1))
        h2 = int(splitmix64(np.uint64(h)))
        m = 1 + h2 % 4
        phi = (int(splitmix64(np.uint64(h2))) >> 11) * (2.0 ** -53) * 2.0 * math.pi
        modes.append((m, phi))
    return ks, modes


def kh_ensemble(nsims: int = 64, seed: int = 1204, steps: int = 100, precision="fp32",
                kmin: int = 4, kmax: int = 32) -> Workload:
    """Independent 2-D KH runs on [0,1]x[-0.5,0.5] (periodic x, outflow y),
    N_k = 16 k_k cells per side with k_k drawn from the seed."""
    ks, modes = kh_sizes(nsims, seed, kmin, kmax)
    sims = [SimDesc(lo=(0.0, -0.5, 0.0), hi=(1.0, 0.5, 1.0), nbase=(k, k, 1),
                    bc=(("periodic", "periodic"), ("outflow", "outflow"),
                        ("periodic", "periodic"))) for k in ks]
    keys = np.concatenate([base_keys(i, s.nbase, 2) for i, s in enumerate(sims)])
    return Workload(name=f"kh_ensemble_{nsims}", ndim=2, sims=sims, keys=keys, ic=_kh_ic,
                    steps=steps, precision=precision, seed=seed, extra={"modes": modes})


def _alfven_ic(wl, sim, lv, x, y, z, gidx):
    A = wl.extra["amp"]
    rho0, p0, B0 = 1.0, 0.1, 1.0
    kx, ky = 2.0 * math.pi, 2.0 * math.pi
    ph = np.sin(kx * x + ky * y)
    s = 1.0 / math.sqrt(2.0)
    return [rho0, 0.0, 0.0, A * ph, B0 * s, B0 * s, -A * math.sqrt(rho0) * ph, p0, 0.0]


def alfven2d(nbase: int, amp: float = 1e-6, scheme="lf", limiter="minmod") -> Workload:
    """Linear Alfven wave along k = 2 pi (1, 1) with B0 parallel to k on the
    periodic unit square; v_z and B_z carry the perturbation."""
    sims = [_unit_square(nbase)]
    return Workload(name=f"alfven_{16 * nbase}", ndim=2, sims=sims,
                    keys=base_keys(0, sims[0].nbase, 2), ic=_alfven_ic, scheme=scheme,
                    limiter=limiter, extra={"amp": amp})


def alfven_exact_vz(x, y, t, amp=1e-6):
    """Exact v_z of the linear Alfven wave: a shift by v_A t along k-hat (v_A = 1)."""
    k = 2.0 * math.pi
    return amp * np.sin(k * x + k * y - k * math.sqrt(2.0) * t)


def advection1d_ic(x, t=0.0):
    """Density of the 1-D advection accuracy test (rho = (sin 2 pi x + 2)/3, v = 1)."""
    return (np.sin(2.0 * math.pi * (x - t)) + 2.0) / 3.0


def advection2d_ic(x, y, t=0.0):
    """Density of the 2-D oblique advection test, v = (1, sqrt 3)."""
    xs, ys = x - t, y - math.sqrt(3.0) * t
    return (np.sin(2.0 * math.pi * (xs + ys / math.sqrt(3.0)) + math.pi / 2.0) + 2.0) / 3.0


# ---------------------------------------------------------------- registry
def by_name(name: str, **kw) -> Workload:
    table = {
        "orszag_tang": orszag_tang,
        "blast3d": blast3d,
        "harris3d": harris3d,
        "kh_ensemble": kh_ensemble,
    }
    return table[name](**kw)
