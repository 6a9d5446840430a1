"""ctypes binding of libmap.so (include/map.h): same names, argument
marshalling only.  Every stage of the block update runs in the HIP kernels of
the library; if the library is not built this module raises on import of any
entry point -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmap.so")

MAP_OK, MAP_EINVAL, MAP_ETREE, MAP_ENOMEM, MAP_EHIP, MAP_ENONFINITE, MAP_ENEGPRESSURE, MAP_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
MAP_FP64, MAP_FP32_MIXED = 0, 1
MAP_LF, MAP_MMC, MAP_WENO = 0, 1, 2
MAP_MINMOD, MAP_VANLEER, MAP_PAPER_PHI = 0, 1, 2
MAP_GLM_PAPER, MAP_GLM_FASTSPEED = 0, 1
MAP_BC_PERIODIC, MAP_BC_OUTFLOW = 0, 1
MAP_LAUNCH_BATCHED, MAP_LAUNCH_PER_BLOCK = 0, 1
MAP_EST_VAR, MAP_EST_BMAG = 0, 1
MAP_RUSANOV, MAP_HLLC = 0, 1
MAP_COND_OFF, MAP_COND_ISO, MAP_COND_FIELD = 0, 1, 2

SCHEMES = {"lf": MAP_LF, "mmc": MAP_MMC, "weno": MAP_WENO}
LIMITERS = {"minmod": MAP_MINMOD, "vanleer": MAP_VANLEER, "paper": MAP_PAPER_PHI}
GLM = {"paper": MAP_GLM_PAPER, "fastspeed": MAP_GLM_FASTSPEED}
BC = {"periodic": MAP_BC_PERIODIC, "outflow": MAP_BC_OUTFLOW}
PRECISION = {"fp64": MAP_FP64, "fp32": MAP_FP32_MIXED}
RIEMANN = {"rusanov": MAP_RUSANOV, "hllc": MAP_HLLC}
COND = {"off": MAP_COND_OFF, "iso": MAP_COND_ISO, "field": MAP_COND_FIELD}

EXPORTS = ["map_init_blocks", "map_query", "map_neighbors", "map_fill_selection", "map_bind_workspace",
           "map_prim_to_cons", "map_fill_ghosts", "map_restrict", "map_prolong", "map_cfl_dt",
           "map_step", "map_reflux", "map_conduct", "map_totals", "map_totals_static",
           "map_status_flags", "map_advance",
           "map_graph_run", "map_set_launch", "map_get_launch", "map_set_launch_config",
           "map_autotune", "map_estimate", "map_regrid", "map_regrid_interval",
           "map_remap", "map_last_error", "map_destroy"]


class MapError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"map status {status}: {msg}")
        self.status = status


class map_params(C.Structure):
    _fields_ = [("ndim", C.c_int), ("precision", C.c_int), ("scheme", C.c_int),
                ("limiter", C.c_int), ("glm_mode", C.c_int), ("eglm_sources", C.c_int),
                ("riemann", C.c_int), ("cond_mode", C.c_int), ("cond_max_sub", C.c_int),
                ("gamma", C.c_double), ("cfl", C.c_double), ("glm_cd", C.c_double),
                ("glm_cr", C.c_double), ("eta", C.c_double), ("kappa0", C.c_double),
                ("kappa_exp", C.c_double)]


class map_sim_desc(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("nbase", C.c_int * 3),
                ("bc", (C.c_int * 2) * 3)]


class map_block_key(C.Structure):
    _fields_ = [("sim", C.c_int), ("level", C.c_int), ("ix", C.c_int), ("iy", C.c_int),
                ("iz", C.c_int)]


class map_dt(C.Structure):
    _fields_ = [("dt", C.c_double), ("ch", C.c_double), ("damp", C.c_double),
                ("alpha", C.c_double), ("dt_sub", C.c_double), ("nsub", C.c_int),
                ("reserved", C.c_int)]


DT_WORDS = C.sizeof(map_dt) // 8  # float64 words per record


class map_sizes(C.Structure):
    _fields_ = [("state_bytes", C.c_size_t), ("workspace_bytes", C.c_size_t),
                ("nblocks", C.c_int), ("nleaves", C.c_int), ("nsims", C.c_int),
                ("max_level", C.c_int), ("tile_cells", C.c_int), ("nvar", C.c_int),
                ("n_prolong_items", C.c_int), ("n_reflux_blocks", C.c_int),
                ("n_face_buffers", C.c_int)]


class map_launch(C.Structure):
    _fields_ = [("mode", C.c_int), ("grid_step", C.c_int), ("grid_fill", C.c_int),
                ("step_shape", C.c_int), ("restrict_split", C.c_int),
                ("step_blocks_per_group", C.c_int), ("cfl_in_update", C.c_int),
                ("cfl_in_update_on", C.c_int)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class map_estimator(C.Structure):
    _fields_ = [("ncrit", C.c_int), ("mode", C.c_int * 4), ("var", C.c_int * 4),
                ("eps", C.c_double * 4), ("filt", C.c_double), ("bias", C.c_double),
                ("ratio", C.c_double), ("xi", C.c_double)]


class map_regrid_params(C.Structure):
    _fields_ = [("tau_refine", C.c_double), ("tau_coarsen", C.c_double), ("max_level", C.c_int)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1204_5849_amd.build` (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp, st = C.c_void_p, C.c_int
        L.map_init_blocks.argtypes = [C.POINTER(vp), C.POINTER(map_params), C.c_int,
                                      C.POINTER(map_sim_desc), C.c_int, C.POINTER(map_block_key)]
        L.map_query.argtypes = [vp, C.POINTER(map_sizes), C.POINTER(C.c_int32)]
        L.map_neighbors.argtypes = [vp, C.POINTER(C.c_int32)]
        L.map_fill_selection.argtypes = [vp, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_uint32),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int)]
        L.map_bind_workspace.argtypes = [vp, vp, C.c_size_t, vp]
        L.map_prim_to_cons.argtypes = [vp, vp, vp]
        L.map_fill_ghosts.argtypes = [vp, vp, vp]
        L.map_restrict.argtypes = [vp, vp, vp]
        L.map_prolong.argtypes = [vp, vp, vp, C.c_int, vp]
        L.map_cfl_dt.argtypes = [vp, vp, vp, vp]
        L.map_step.argtypes = [vp, vp, vp, vp, vp]
        L.map_reflux.argtypes = [vp, vp, vp, vp]
        L.map_conduct.argtypes = [vp, vp, vp, vp]
        L.map_totals.argtypes = [vp, vp, vp, vp]
        L.map_totals_static.argtypes = [vp, vp, vp, vp]
        L.map_status_flags.argtypes = [vp, C.POINTER(C.c_uint64), vp]
        L.map_advance.argtypes = [vp, vp, vp, C.c_int, vp]
        L.map_graph_run.argtypes = [vp, vp, vp, C.c_int, vp]
        L.map_set_launch.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.map_autotune.argtypes = [vp, vp, C.POINTER(C.c_int), vp]
        L.map_get_launch.argtypes = [vp, C.POINTER(map_launch)]
        L.map_set_launch_config.argtypes = [vp, C.POINTER(map_launch)]
        L.map_estimate.argtypes = [vp, vp, C.POINTER(map_estimator), vp, vp]
        L.map_regrid.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(map_regrid_params),
                                 C.POINTER(map_block_key), C.c_int, C.POINTER(C.c_int)]
        L.map_remap.argtypes = [vp, vp, vp, vp, vp]
        L.map_regrid_interval.argtypes = [vp, C.POINTER(map_dt), C.c_double,
                                          C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.map_last_error.restype = C.c_char_p
        L.map_last_error.argtypes = []
        L.map_destroy.argtypes = [vp]
        L.map_destroy.restype = None
        for name in EXPORTS:
            if name not in ("map_last_error", "map_destroy"):
                getattr(L, name).restype = st
        _lib = L
    return _lib


def check(status: int):
    if status != MAP_OK:
        raise MapError(status, lib().map_last_error().decode(errors="replace"))
    return status


def _p(x):
    """Device pointer of a torch tensor, or an int / None."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return int(x)


# ---------------------------------------------------------------- thin wrappers
def make_params(ndim, precision="fp64", scheme="lf", limiter="minmod", glm_mode="paper",
                eglm_sources=True, gamma=5.0 / 3.0, cfl=0.4, cd=0.18, cr=0.18, eta=0.0,
                riemann="rusanov", cond="off", cond_max_sub=8, kappa0=0.0, kappa_exp=2.5):
    p = map_params()
    p.ndim = ndim
    p.precision = PRECISION.get(precision, precision)
    p.scheme = SCHEMES.get(scheme, scheme)
    p.limiter = LIMITERS.get(limiter, limiter)
    p.glm_mode = GLM.get(glm_mode, glm_mode)
    p.eglm_sources = int(bool(eglm_sources))
    p.riemann = RIEMANN.get(riemann, riemann)
    p.cond_mode = COND.get(cond, cond)
    p.cond_max_sub = cond_max_sub
    p.kappa0, p.kappa_exp = kappa0, kappa_exp
    p.gamma, p.cfl, p.glm_cd, p.glm_cr, p.eta = gamma, cfl, cd, cr, eta
    return p


def make_sims(sims):
    arr = (map_sim_desc * len(sims))()
    for i, s in enumerate(sims):
        for d in range(3):
            arr[i].lo[d] = s.lo[d]
            arr[i].hi[d] = s.hi[d]
            arr[i].nbase[d] = s.nbase[d]
            for side in range(2):
                arr[i].bc[d][side] = BC[s.bc[d][side]]
    return arr


def make_keys(keys):
    import numpy as np
    keys = np.ascontiguousarray(np.asarray(keys, dtype=np.int32))
    arr = (map_block_key * len(keys))()
    C.memmove(arr, keys.ctypes.data, keys.nbytes)
    return arr


def map_init_blocks(params, sims, keys):
    ctx = C.c_void_p()
    s = make_sims(sims)
    k = make_keys(keys)
    check(lib().map_init_blocks(C.byref(ctx), C.byref(params), len(sims), s, len(keys), k))
    return ctx


def map_query(ctx):
    import numpy as np
    sz = map_sizes()
    check(lib().map_query(ctx, C.byref(sz), None))
    slots = np.zeros(sz.nblocks, dtype=np.int32)
    check(lib().map_query(ctx, C.byref(sz), slots.ctypes.data_as(C.POINTER(C.c_int32))))
    return sz, slots


def map_neighbors(ctx, nblocks):
    import numpy as np
    out = np.zeros((nblocks, 27), dtype=np.int32)
    check(lib().map_neighbors(ctx, out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


def map_fill_selection(ctx):
    """(parent input indices, direction masks, boxes [n, 6]) of the cycle's fill."""
    import numpy as np
    n = C.c_int()
    check(lib().map_fill_selection(ctx, 0, None, None, None, C.byref(n)))
    par = np.zeros(n.value, dtype=np.int32)
    dirs = np.zeros(n.value, dtype=np.uint32)
    box = np.zeros((n.value, 6), dtype=np.int32)
    check(lib().map_fill_selection(ctx, n.value, par.ctypes.data_as(C.POINTER(C.c_int32)),
                                   dirs.ctypes.data_as(C.POINTER(C.c_uint32)),
                                   box.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n)))
    return par, dirs, box


def map_bind_workspace(ctx, ws, nbytes, stream):
    check(lib().map_bind_workspace(ctx, _p(ws), nbytes, _p(stream)))


def map_prim_to_cons(ctx, U, stream):
    check(lib().map_prim_to_cons(ctx, _p(U), _p(stream)))


def map_fill_ghosts(ctx, U, stream):
    check(lib().map_fill_ghosts(ctx, _p(U), _p(stream)))


def map_restrict(ctx, U, stream):
    check(lib().map_restrict(ctx, _p(U), _p(stream)))


def map_prolong(ctx, U, slots_dev, n, stream):
    check(lib().map_prolong(ctx, _p(U), _p(slots_dev), n, _p(stream)))


def map_cfl_dt(ctx, U, dt_dev, stream):
    check(lib().map_cfl_dt(ctx, _p(U), _p(dt_dev), _p(stream)))


def map_step(ctx, Uin, Uout, dt_dev, stream):
    check(lib().map_step(ctx, _p(Uin), _p(Uout), _p(dt_dev), _p(stream)))


def map_reflux(ctx, U, dt_dev, stream):
    check(lib().map_reflux(ctx, _p(U), _p(dt_dev), _p(stream)))


def map_conduct(ctx, U, dt_dev, stream):
    check(lib().map_conduct(ctx, _p(U), _p(dt_dev), _p(stream)))


def map_totals(ctx, U, out_dev, stream):
    check(lib().map_totals(ctx, _p(U), _p(out_dev), _p(stream)))


def map_totals_static(ctx, U, out_dev, stream):
    check(lib().map_totals_static(ctx, _p(U), _p(out_dev), _p(stream)))


def map_status_flags(ctx, stream):
    """Returns (status, counters[4]) without raising on the two state errors."""
    arr = (C.c_uint64 * 4)()
    st = lib().map_status_flags(ctx, arr, _p(stream))
    if st not in (MAP_OK, MAP_ENONFINITE, MAP_ENEGPRESSURE):
        check(st)
    return st, [int(v) for v in arr]


def map_advance(ctx, U, dt_dev, nsteps, stream):
    check(lib().map_advance(ctx, _p(U), _p(dt_dev), nsteps, _p(stream)))


def map_graph_run(ctx, U, dt_dev, nsteps, stream):
    check(lib().map_graph_run(ctx, _p(U), _p(dt_dev), nsteps, _p(stream)))


def map_set_launch(ctx, mode, grid_step=0, grid_fill=0):
    check(lib().map_set_launch(ctx, mode, grid_step, grid_fill))


def map_autotune(ctx, U, stream):
    arr = (C.c_int * 2)()
    check(lib().map_autotune(ctx, _p(U), arr, _p(stream)))
    return int(arr[0]), int(arr[1])


def map_get_launch(ctx) -> dict:
    out = map_launch()
    check(lib().map_get_launch(ctx, C.byref(out)))
    return out.as_dict()


# map_launch fields that map_get_launch reports and map_set_launch_config ignores
LAUNCH_READ_ONLY = ("step_blocks_per_group", "cfl_in_update_on")


def map_set_launch_config(ctx, cfg: dict):
    """Set the launch settings named in `cfg`, keeping the others (read-only
    fields in `cfg` are ignored)."""
    x = map_launch()
    cur = map_get_launch(ctx)
    cur.update({k: v for k, v in cfg.items() if k not in LAUNCH_READ_ONLY})
    for k, _ in map_launch._fields_:
        setattr(x, k, int(cur[k]))
    check(lib().map_set_launch_config(ctx, C.byref(x)))


def make_estimator(criteria, filt=0.05, bias=0.6, ratio=2.0, xi=0.0):
    """criteria: up to 4 tuples (mode, var, eps) with mode "var" (conserved
    variable index var) or "bmag" (|B|)."""
    e = map_estimator()
    e.ncrit = len(criteria)
    for i, (mode, var, eps) in enumerate(criteria):
        e.mode[i] = {"var": MAP_EST_VAR, "bmag": MAP_EST_BMAG}.get(mode, mode)
        e.var[i] = var
        e.eps[i] = eps
    e.filt, e.bias, e.ratio, e.xi = filt, bias, ratio, xi
    return e


def map_estimate(ctx, U, est, err_dev, stream):
    check(lib().map_estimate(ctx, _p(U), C.byref(est), _p(err_dev), _p(stream)))


def map_regrid_interval(ctx, dt_host, c_r):
    """(dtr per simulation, steps per simulation) from host dt records
    (float64 numpy [nsims, DT_WORDS])."""
    import numpy as np
    rec = np.ascontiguousarray(np.asarray(dt_host, dtype=np.float64))
    ns = rec.shape[0]
    dtr = np.zeros(ns)
    steps = np.zeros(ns, dtype=np.int32)
    check(lib().map_regrid_interval(ctx, rec.ctypes.data_as(C.POINTER(map_dt)), float(c_r),
                                    dtr.ctypes.data_as(C.POINTER(C.c_double)),
                                    steps.ctypes.data_as(C.POINTER(C.c_int))))
    return dtr, steps


def map_regrid(ctx, err_host, tau_refine, tau_coarsen, max_level):
    """New keys (int32 [n, 5], sorted) from per-slot estimates (float64)."""
    import numpy as np
    err = np.ascontiguousarray(np.asarray(err_host, dtype=np.float64))
    rp = map_regrid_params(tau_refine, tau_coarsen, max_level)
    n = C.c_int(0)
    st = lib().map_regrid(ctx, err.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rp), None, 0,
                          C.byref(n))
    if st not in (MAP_OK, MAP_ENOMEM):
        check(st)
    out = (map_block_key * max(n.value, 1))()
    check(lib().map_regrid(ctx, err.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rp), out,
                           n.value, C.byref(n)))
    keys = np.frombuffer(out, dtype=np.int32, count=5 * n.value).reshape(n.value, 5).copy()
    return keys


def map_remap(dst_ctx, U_dst, src_ctx, U_src, stream):
    check(lib().map_remap(dst_ctx, _p(U_dst), src_ctx, _p(U_src), _p(stream)))


def map_destroy(ctx):
    if ctx:
        lib().map_destroy(ctx)
