"""FP64 CPU oracle of the MAP block update -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and its
Python binding) never imports, links or executes anything here, and this
package never touches the HIP library: the two share nothing but the seeded
input generator in ``paper_1204_5849_amd.workloads``.

The arithmetic lives in ``oracle.c`` (plain C, FP64, ``-O2
-ffp-contract=off``); this module only builds it and marshals arguments.
Functions whose results are not pinned by a test against the paper or the
mathematics are listed as "parity unpinned" in the design notes; every
function exported here has at least one pin in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

MHD, SCALAR = 0, 1
LF, MMC, WENO = 0, 1, 2
MINMOD, VANLEER, PAPER_PHI = 0, 1, 2
GLM_PAPER, GLM_FASTSPEED = 0, 1
BC_PERIODIC, BC_OUTFLOW = 0, 1
RUSANOV, HLLC = 0, 1
COND_OFF, COND_ISO, COND_FIELD = 0, 1, 2

_SCHEMES = {"lf": LF, "mmc": MMC, "weno": WENO}
_LIMITERS = {"minmod": MINMOD, "vanleer": VANLEER, "paper": PAPER_PHI}
_GLM = {"paper": GLM_PAPER, "fastspeed": GLM_FASTSPEED}
_BC = {"periodic": BC_PERIODIC, "outflow": BC_OUTFLOW}
_RIEMANN = {"rusanov": RUSANOV, "hllc": HLLC}
_COND = {"off": COND_OFF, "iso": COND_ISO, "field": COND_FIELD}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, FP64, no contraction)."""
    src = os.path.join(HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                               "-fopenmp", "-Wall", "-Wno-unused-function", "-shared", "-fPIC",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("ndim", C.c_int), ("physics", C.c_int), ("scheme", C.c_int),
                ("limiter", C.c_int), ("glm_mode", C.c_int), ("eglm_sources", C.c_int),
                ("riemann", C.c_int), ("cond_mode", C.c_int), ("cond_max_sub", C.c_int),
                ("gamma", C.c_double), ("cfl", C.c_double), ("cd", C.c_double),
                ("cr", C.c_double), ("eta", C.c_double), ("kappa0", C.c_double),
                ("kappa_exp", C.c_double), ("adv", C.c_double * 3)]


class DtRec(C.Structure):
    _fields_ = [("dt", C.c_double), ("ch", C.c_double), ("damp", C.c_double),
                ("alpha", C.c_double), ("dt_sub", C.c_double), ("nsub", C.c_int),
                ("reserved", C.c_int)]

    def as_tuple(self):
        return (self.dt, self.ch, self.damp, self.alpha)


class Sim(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("nbase", C.c_int * 3),
                ("bc", (C.c_int * 2) * 3)]


class Key(C.Structure):
    _fields_ = [("sim", C.c_int), ("level", C.c_int), ("ix", C.c_int), ("iy", C.c_int),
                ("iz", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(Params)
        ip = C.POINTER(C.c_int)
        lp = C.POINTER(C.c_long)
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_nvar.argtypes = [pp]
        L.orc_pressure.argtypes = [pp, dp]
        L.orc_pressure.restype = C.c_double
        L.orc_flux.argtypes = [pp, dp, C.c_int, C.c_double, dp]
        L.orc_speed.argtypes = [pp, dp, C.c_int]
        L.orc_speed.restype = C.c_double
        L.orc_limiter.argtypes = [C.c_int, C.c_double, C.c_double]
        L.orc_limiter.restype = C.c_double
        L.orc_face_flux.argtypes = [pp, dp, dp, C.c_int, C.c_double, dp]
        L.orc_hllc_fan.argtypes = [pp, dp, dp, C.c_int, C.c_double, dp, dp, dp]
        L.orc_weno_face.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_weno_face.restype = C.c_double
        L.orc_prim_to_cons.argtypes = [pp, dp, C.c_long]
        L.orc_step_tile.argtypes = [pp, dp, dp, ip, C.POINTER(DtRec), dp, dp, lp]
        L.orc_lf_states.argtypes = [pp, dp, dp, ip, C.POINTER(DtRec), dp, dp, dp, lp]
        L.orc_eglm_source.argtypes = [pp, dp, dp, ip, dp]
        L.orc_resistive.argtypes = [pp, dp, dp, ip, dp]
        L.orc_tile_maxspeed.argtypes = [pp, dp, ip]
        L.orc_tile_maxspeed.restype = C.c_double
        L.orc_make_dtrec.argtypes = [pp, C.c_double, C.c_double, C.c_double, C.POINTER(DtRec)]
        L.orc_tile_cond_rate.argtypes = [pp, dp, ip]
        L.orc_tile_cond_rate.restype = C.c_double
        L.orc_conduct_tile.argtypes = [pp, dp, dp, ip, C.c_double, dp, dp]
        L.orc_amr_conduct.argtypes = [C.c_void_p, C.POINTER(DtRec)]
        L.orc_grid_fill.argtypes = [pp, dp, ip, ip]
        L.orc_grid_run.argtypes = [pp, dp, dp, ip, ip, C.c_int, dp, lp]
        L.orc_amr_new.argtypes = [pp, C.c_int, C.c_int, C.POINTER(Sim), C.c_int, C.POINTER(Key)]
        L.orc_amr_new.restype = C.c_void_p
        L.orc_amr_free.argtypes = [C.c_void_p]
        L.orc_amr_state.argtypes = [C.c_void_p]
        L.orc_amr_state.restype = dp
        L.orc_amr_tile_cells.argtypes = [C.c_void_p]
        L.orc_amr_is_leaf.argtypes = [C.c_void_p, C.c_int]
        for name in ("orc_amr_prim_to_cons", "orc_amr_fill", "orc_amr_restrict"):
            getattr(L, name).argtypes = [C.c_void_p]
        L.orc_amr_prolong_block.argtypes = [C.c_void_p, C.c_int]
        L.orc_amr_cfl.argtypes = [C.c_void_p, C.POINTER(DtRec)]
        L.orc_amr_step.argtypes = [C.c_void_p, C.POINTER(DtRec)]
        L.orc_amr_reflux.argtypes = [C.c_void_p, C.POINTER(DtRec)]
        L.orc_amr_totals.argtypes = [C.c_void_p, dp]
        L.orc_amr_run.argtypes = [C.c_void_p, C.c_int, C.POINTER(DtRec)]
        L.orc_amr_counters.argtypes = [C.c_void_p, lp]
        L.orc_estimate.argtypes = [pp, dp, ip, C.c_int, C.c_int, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_estimate.restype = C.c_double
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the block-tree loops (default 1); any count gives the
    one-thread result bit for bit."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int))


def make_params(ndim=2, physics=MHD, scheme="lf", limiter="minmod", glm_mode="paper",
                eglm_sources=True, gamma=5.0 / 3.0, cfl=0.4, cd=0.18, cr=0.18, eta=0.0,
                adv=(0.0, 0.0, 0.0), riemann="rusanov", cond="off", cond_max_sub=8,
                kappa0=0.0, kappa_exp=2.5) -> Params:
    p = Params()
    p.ndim = ndim
    p.physics = physics
    p.scheme = _SCHEMES.get(scheme, scheme)
    p.limiter = _LIMITERS.get(limiter, limiter)
    p.glm_mode = _GLM.get(glm_mode, glm_mode)
    p.eglm_sources = int(bool(eglm_sources))
    p.riemann = _RIEMANN.get(riemann, riemann)
    p.cond_mode = _COND.get(cond, cond)
    p.cond_max_sub = cond_max_sub
    p.kappa0, p.kappa_exp = kappa0, kappa_exp
    p.gamma, p.cfl, p.cd, p.cr, p.eta = gamma, cfl, cd, cr, eta
    for i in range(3):
        p.adv[i] = adv[i]
    return p


def params_from_workload(w) -> Params:
    return make_params(ndim=w.ndim, scheme=w.scheme, limiter=w.limiter, glm_mode=w.glm_mode,
                       eglm_sources=w.eglm_sources, gamma=w.gamma, cfl=w.cfl, cd=w.cd,
                       cr=w.cr, eta=w.eta, riemann=w.riemann, cond=w.cond,
                       cond_max_sub=w.cond_max_sub, kappa0=w.kappa0, kappa_exp=w.kappa_exp)


def nvar(p: Params) -> int:
    return 9 if p.physics == MHD else 1


# ---------------------------------------------------------------- pointwise
def pressure(p, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_pressure(C.byref(p), _dp(u))


def flux(p, u, dim, ch=0.0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.zeros(nvar(p))
    lib().orc_flux(C.byref(p), _dp(u), dim, ch, _dp(f))
    return f


def speed(p, u, dim):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_speed(C.byref(p), _dp(u), dim)


def limiter(kind, a, b):
    kind = _LIMITERS.get(kind, kind)
    return lib().orc_limiter(kind, float(a), float(b))


def face_flux(p, L, R, dim, ch=0.0):
    """Face flux (Rusanov or HLLC, as p.riemann selects) between two states."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    out = np.zeros(nvar(p))
    lib().orc_face_flux(C.byref(p), _dp(L), _dp(R), dim, float(ch), _dp(out))
    return out


def hllc_fan(p, L, R, dim, ch=0.0):
    """HLLC fan of a face: ((S_L, S_M, S_R), star state left, star state right)."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    S, a, b = np.zeros(3), np.zeros(9), np.zeros(9)
    lib().orc_hllc_fan(C.byref(p), _dp(L), _dp(R), dim, float(ch), _dp(S), _dp(a), _dp(b))
    return S, a, b


def weno_face(um, u0, up, side):
    """WENO face state from three cells: side 0 = u^-_{i+1/2}, 1 = u^+_{i-1/2}."""
    return lib().orc_weno_face(float(um), float(u0), float(up), int(side))


def prim_to_cons(p, w):
    """w: [9, ...] primitive array (rho, v, B, p, psi); returns conserved copy."""
    w = np.array(w, dtype=np.float64, order="C")
    nc = w[0].size
    lib().orc_prim_to_cons(C.byref(p), _dp(w.reshape(w.shape[0], -1)), nc)
    return w


def dtrec(p, alpha, dxmin, kmax=0.0) -> DtRec:
    r = DtRec()
    lib().orc_make_dtrec(C.byref(p), alpha, dxmin, kmax, C.byref(r))
    return r


def make_dtrec(dt, ch=0.0, damp=1.0, alpha=0.0) -> DtRec:
    r = DtRec()
    r.dt, r.ch, r.damp, r.alpha = dt, ch, damp, alpha
    return r


# ---------------------------------------------------------------- tiles
def tile_shape(p, n):
    """Padded tile shape [nvar, pz, py, px] for interior sizes n=(nx, ny, nz)."""
    nd = p.ndim
    px, py = n[0] + 4, n[1] + 4
    pz = n[2] + 4 if nd == 3 else 1
    return (nvar(p), pz, py, px)


def interior(p, u):
    """View of the interior of a padded tile array [..., nv, pz, py, px]."""
    if p.ndim == 3:
        return u[..., 2:-2, 2:-2, 2:-2]
    return u[..., :, 2:-2, 2:-2]


def _n3(p, n):
    n = list(n) + [1] * (3 - len(n))
    if p.ndim == 2:
        n[2] = 1
    return np.array(n, dtype=np.int32)


def step_tile(p, dx, u, n, rec: DtRec, want_faces=False):
    n3 = _n3(p, n)
    u = np.ascontiguousarray(u, dtype=np.float64)
    nv = nvar(p)
    nint = int(np.prod(n3))
    unew = np.zeros(nv * nint)
    dxa = np.array(list(dx) + [1.0] * (3 - len(dx)), dtype=np.float64)
    if want_faces:
        T = [int(np.prod([n3[j] for j in range(3) if j != d])) for d in range(p.ndim)]
        ff = np.zeros(sum(2 * nv * t for t in T))
        ffp = _dp(ff)
    else:
        ff, ffp = None, None
    cnt = np.zeros(4, dtype=np.int64)
    n3c, n3p = _ip(n3)
    lib().orc_step_tile(C.byref(p), _dp(dxa), _dp(u), n3p, C.byref(rec), _dp(unew), ffp,
                        cnt.ctypes.data_as(C.POINTER(C.c_long)))
    shape = (nv, n3[2], n3[1], n3[0])
    return unew.reshape(shape), ff, cnt


def lf_states(p, dx, u, n, rec: DtRec):
    """Intermediate states of the LF scheme on a padded tile: (u~ [nv, pz, py,
    px], slopes [ndim, nv, pz, py, px], face states [ndim, 2, nv, pz, py, px]
    (left, right; face c+1/2 stored at cell c), counters)."""
    n3 = _n3(p, n)
    u = np.ascontiguousarray(u, dtype=np.float64)
    shape = tile_shape(p, n3)
    nd = p.ndim
    ut = np.zeros(shape)
    sl = np.zeros((nd,) + shape)
    lr = np.zeros((nd, 2) + shape)
    dxa = np.array(list(dx) + [1.0] * (3 - len(dx)), dtype=np.float64)
    cnt = np.zeros(4, dtype=np.int64)
    n3c, n3p = _ip(n3)
    lib().orc_lf_states(C.byref(p), _dp(dxa), _dp(u), n3p, C.byref(rec), _dp(ut), _dp(sl),
                        _dp(lr), cnt.ctypes.data_as(C.POINTER(C.c_long)))
    return ut, sl, lr, cnt


def eglm_source(p, dx, u, n):
    n3 = _n3(p, n)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(nvar(p) * int(np.prod(n3)))
    dxa = np.array(list(dx) + [1.0] * (3 - len(dx)), dtype=np.float64)
    n3c, n3p = _ip(n3)
    lib().orc_eglm_source(C.byref(p), _dp(dxa), _dp(u), n3p, _dp(out))
    return out.reshape(nvar(p), n3[2], n3[1], n3[0])


def resistive(p, dx, u, n):
    n3 = _n3(p, n)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(nvar(p) * int(np.prod(n3)))
    dxa = np.array(list(dx) + [1.0] * (3 - len(dx)), dtype=np.float64)
    n3c, n3p = _ip(n3)
    lib().orc_resistive(C.byref(p), _dp(dxa), _dp(u), n3p, _dp(out))
    return out.reshape(nvar(p), n3[2], n3[1], n3[0])


def tile_maxspeed(p, u, n):
    n3c, n3p = _ip(_n3(p, n))
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_tile_maxspeed(C.byref(p), _dp(u), n3p)


def tile_cond_rate(p, u, n):
    """Largest kappa T / p over the interior of a padded tile."""
    n3c, n3p = _ip(_n3(p, n))
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_tile_cond_rate(C.byref(p), _dp(u), n3p)


def conduct_tile(p, dx, u, n, dt_sub, want_faces=False):
    """One conduction sub-step on a padded tile: (new interior energy
    [nz, ny, nx], face fluxes or None)."""
    n3 = _n3(p, n)
    n3c, n3p = _ip(n3)
    u = np.ascontiguousarray(u, dtype=np.float64)
    dxa = np.ascontiguousarray(list(dx) + [1.0] * (3 - len(dx)), dtype=np.float64)[:3]
    enew = np.zeros((n3[2], n3[1], n3[0]))
    ff = None
    if want_faces:
        nf = 0
        for d in range(p.ndim):
            t1, t2 = (1 if d == 0 else 0), (1 if d == 2 else 2)
            nf += 2 * nvar(p) * int(n3[t1]) * int(n3[t2])
        ff = np.zeros(nf)
    lib().orc_conduct_tile(C.byref(p), _dp(dxa), _dp(u), n3p, float(dt_sub), _dp(enew),
                           _dp(ff) if ff is not None else None)
    return enew, ff


def _bc_arr(bc):
    out = np.zeros((3, 2), dtype=np.int32)
    for d in range(3):
        for s in range(2):
            v = bc[d][s] if d < len(bc) else "periodic"
            out[d, s] = _BC.get(v, v)
    return out


def grid_fill(p, u, n, bc):
    n3c, n3p = _ip(_n3(p, n))
    bcc, bcp = _ip(_bc_arr(bc))
    lib().orc_grid_fill(C.byref(p), _dp(u), n3p, bcp)


def grid_run(p, dx, u, n, bc, nsteps):
    """Advance a monolithic padded grid in place; returns (dt per step, counters)."""
    n3c, n3p = _ip(_n3(p, n))
    bcc, bcp = _ip(_bc_arr(bc))
    dxa = np.array(list(dx) + [1.0] * (3 - len(dx)), dtype=np.float64)
    trace = np.zeros(max(nsteps, 1))
    cnt = np.zeros(4, dtype=np.int64)
    lib().orc_grid_run(C.byref(p), _dp(dxa), _dp(u), n3p, bcp, nsteps, _dp(trace),
                       cnt.ctypes.data_as(C.POINTER(C.c_long)))
    return trace[:nsteps], cnt


def estimate(p, u, n, mode, k_var=0, eps=1e-12, filt=0.05, bias=0.6, ratio=2.0, xi=0.0,
             level=1):
    n3c, n3p = _ip(_n3(p, n))
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_estimate(C.byref(p), _dp(u), n3p, mode, k_var, eps, filt, bias, ratio,
                              xi, level)


# ---------------------------------------------------------------- block tree
def make_sims(sims):
    arr = (Sim * len(sims))()
    for i, s in enumerate(sims):
        for d in range(3):
            arr[i].lo[d] = s.lo[d]
            arr[i].hi[d] = s.hi[d]
            arr[i].nbase[d] = s.nbase[d]
            for side in range(2):
                arr[i].bc[d][side] = _BC[s.bc[d][side]]
    return arr


def make_keys(keys):
    keys = np.asarray(keys, dtype=np.int32)
    arr = (Key * len(keys))()
    C.memmove(arr, np.ascontiguousarray(keys).ctypes.data, keys.nbytes)
    return arr


class Amr:
    """Block tree in the caller's key order; state is [nblocks, nvar, pz, py, px]."""

    def __init__(self, p: Params, n: int, sims, keys):
        self.p = p
        self.n = n
        self.keys = np.ascontiguousarray(np.asarray(keys, dtype=np.int32))
        self.nsims = len(sims)
        self._sims = make_sims(sims)
        self._keys = make_keys(self.keys)
        self.h = lib().orc_amr_new(C.byref(p), n, len(sims), self._sims, len(self.keys),
                                   self._keys)
        P = lib().orc_amr_tile_cells(self.h)
        nv = nvar(p)
        ptr = lib().orc_amr_state(self.h)
        flat = np.ctypeslib.as_array(ptr, shape=(len(self.keys) * nv * P,))
        self.state = flat.reshape((len(self.keys),) + tile_shape(p, (n, n, n)))
        self.leaf = np.array([bool(lib().orc_amr_is_leaf(self.h, b)) for b in range(len(self.keys))])

    def __del__(self):
        # (at interpreter exit the module's globals may already be gone)
        if getattr(self, "h", None) and callable(lib):
            lib().orc_amr_free(self.h)
            self.h = None

    def prim_to_cons(self):
        lib().orc_amr_prim_to_cons(self.h)

    def fill(self):
        lib().orc_amr_fill(self.h)

    def restrict(self):
        lib().orc_amr_restrict(self.h)

    def prolong_block(self, b):
        lib().orc_amr_prolong_block(self.h, int(b))

    def cfl(self):
        r = (DtRec * self.nsims)()
        lib().orc_amr_cfl(self.h, r)
        return r

    def step(self, recs):
        lib().orc_amr_step(self.h, recs)

    def reflux(self, recs):
        lib().orc_amr_reflux(self.h, recs)

    def totals(self):
        out = np.zeros(self.nsims * nvar(self.p))
        lib().orc_amr_totals(self.h, _dp(out))
        return out.reshape(self.nsims, nvar(self.p))

    def run(self, nsteps, trace=False):
        if trace:
            tr = (DtRec * (max(nsteps, 1) * self.nsims))()
            lib().orc_amr_run(self.h, nsteps, tr)
            return np.array([r.as_tuple() for r in tr]).reshape(nsteps, self.nsims, 4)
        lib().orc_amr_run(self.h, nsteps, None)
        return None

    def counters(self):
        out = np.zeros(4, dtype=np.int64)
        lib().orc_amr_counters(self.h, out.ctypes.data_as(C.POINTER(C.c_long)))
        return out

    def interior(self):
        return interior(self.p, self.state)


def load_workload(w, blocks_per_chunk=4096):
    """Build an oracle block tree for a workload: leaves get the seeded
    primitive initial data, then conversion, restriction and ghost fill."""
    p = params_from_workload(w)
    A = Amr(p, w.n, w.sims, w.keys)
    leaves = np.nonzero(A.leaf)[0]
    for s in range(0, len(leaves), blocks_per_chunk):
        idx = leaves[s:s + blocks_per_chunk]
        prim = w.primitive_blocks(idx)  # [len, 9, nz, ny, nx]
        interior(p, A.state)[idx] = prim
    A.prim_to_cons()
    A.restrict()
    A.fill()
    return A
