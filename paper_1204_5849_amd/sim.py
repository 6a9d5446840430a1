"""Device-side driver of one block tree: torch owns the state, workspace and
stream; every stage runs through the C ABI in native.py.

    sim = Simulation(workload, device="cuda:0")
    sim.load_initial()            # primitives -> slots, conversion, restrict, fill
    sim.advance(10)               # or sim.graph_run(10)
    U = sim.state_by_key()        # float64 numpy [nblocks, 9, pz, py, px], input key order
"""
from __future__ import annotations

import numpy as np
import torch

from . import native as N
from .workloads import Workload

NB, NG, PD, NV = 16, 2, 20, 9


class Simulation:
    def __init__(self, wl: Workload, device="cuda:0", stream: torch.cuda.Stream | None = None,
                 precision: str | None = None, launch: str = "batched"):
        if not torch.cuda.is_available():
            raise RuntimeError("Simulation needs a HIP device")
        self.wl = wl
        self.device = torch.device(device)
        self.precision = precision or wl.precision
        self.dtype = torch.float64 if self.precision == "fp64" else torch.float32
        self.params = N.make_params(wl.ndim, precision=self.precision, scheme=wl.scheme,
                                    limiter=wl.limiter, glm_mode=wl.glm_mode, riemann=wl.riemann,
                                    cond=wl.cond, cond_max_sub=wl.cond_max_sub, kappa0=wl.kappa0,
                                    kappa_exp=wl.kappa_exp,
                                    eglm_sources=wl.eglm_sources, gamma=wl.gamma, cfl=wl.cfl,
                                    cd=wl.cd, cr=wl.cr, eta=wl.eta)
        self.stream = stream or torch.cuda.Stream(device=self.device)
        with torch.cuda.device(self.device):
            self.dt = torch.zeros((len(wl.sims), N.DT_WORDS), dtype=torch.float64, device=self.device)
        self._spare = None  # the second pair of buffers of in-place regrids
        self.ctx = N.map_init_blocks(self.params, wl.sims, wl.keys)
        self._plan(wl)
        self._ubuf = torch.zeros(self._u_elems(), dtype=self.dtype, device=self.device)
        self._wsbuf = torch.zeros(self.sizes.workspace_bytes + 256, dtype=torch.uint8,
                                  device=self.device)
        self._bind()
        if launch == "per_block":
            N.map_set_launch(self.ctx, N.MAP_LAUNCH_PER_BLOCK)

    def _plan(self, wl):
        """Sizes and slots of the context's tree."""
        self.wl = wl
        self.sizes, self.slot_of_key = N.map_query(self.ctx)
        self.nslots = self.sizes.nblocks
        self.tile = self.sizes.tile_cells
        pz = PD if wl.ndim == 3 else 1
        self.shape = (self.nslots, NV, pz, PD, PD)

    def _u_elems(self):
        return self.nslots * NV * self.tile

    def _bind(self):
        """State view and workspace of the current context on the current
        buffers (which may be larger than the tree needs)."""
        self.U = self._ubuf[:self._u_elems()].view(self.shape)
        self.ws = self._wsbuf
        torch.cuda.synchronize(self.device)
        self._ws_ptr = (self._wsbuf.data_ptr() + 255) & ~255
        N.map_bind_workspace(self.ctx, self._ws_ptr, self.sizes.workspace_bytes, self.sp)

    @property
    def sp(self):
        return self.stream.cuda_stream

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        # at interpreter exit the binding's module globals may already be
        # gone; the process releases the context then
        destroy = getattr(N, "map_destroy", None) if N is not None else None
        if ctx and destroy is not None:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            destroy(ctx)
            self.ctx = None

    # ---------------------------------------------------------------- data
    def interior_view(self):
        if self.wl.ndim == 3:
            return self.U[:, :, NG:-NG, NG:-NG, NG:-NG]
        return self.U[:, :, :, NG:-NG, NG:-NG]

    def load_initial(self, chunk=2048):
        """Leaves get the seeded primitive data; then conversion to conserved
        variables, restriction of the parents and ghost fill, all on device."""
        leaves = np.nonzero(self.wl.leaf_mask())[0]
        inter = self.interior_view()
        with torch.cuda.stream(self.stream):
            for s in range(0, len(leaves), chunk):
                idx = leaves[s:s + chunk]
                prim = torch.from_numpy(self.wl.primitive_blocks(idx)).to(self.device,
                                                                         non_blocking=False)
                slots = torch.from_numpy(self.slot_of_key[idx].astype(np.int64)).to(self.device)
                inter[slots] = prim.to(self.dtype)
        self.stream.synchronize()
        N.map_prim_to_cons(self.ctx, self.U, self.sp)
        N.map_restrict(self.ctx, self.U, self.sp)
        N.map_fill_ghosts(self.ctx, self.U, self.sp)
        self.stream.synchronize()

    def state_by_key(self, blocks=None) -> np.ndarray:
        """FP64 copy of the state in the caller's key order (optionally a subset)."""
        self.stream.synchronize()
        if blocks is None:
            slots = self.slot_of_key
        else:
            slots = self.slot_of_key[np.asarray(blocks)]
        idx = torch.from_numpy(slots.astype(np.int64)).to(self.device)
        return self.U.index_select(0, idx).to(torch.float64).cpu().numpy()

    # ---------------------------------------------------------------- stages
    def fill(self):
        N.map_fill_ghosts(self.ctx, self.U, self.sp)

    def restrict(self):
        N.map_restrict(self.ctx, self.U, self.sp)

    def cfl(self):
        N.map_cfl_dt(self.ctx, self.U, self.dt, self.sp)
        return self.dt

    def step(self, Uout):
        """One update of every leaf from self.U into Uout (a separate tensor of
        the same shape: the update reads neighbour interiors of self.U)."""
        N.map_step(self.ctx, self.U, Uout, self.dt, self.sp)

    def reflux(self):
        N.map_reflux(self.ctx, self.U, self.dt, self.sp)

    def conduct(self):
        """The conduction subcycle of one step with the current dt records."""
        N.map_conduct(self.ctx, self.U, self.dt, self.sp)

    def totals(self) -> np.ndarray:
        out = torch.zeros((len(self.wl.sims), NV), dtype=torch.float64, device=self.device)
        N.map_totals(self.ctx, self.U, out, self.sp)
        self.stream.synchronize()
        return out.cpu().numpy()

    def advance(self, nsteps):
        N.map_advance(self.ctx, self.U, self.dt, nsteps, self.sp)

    def graph_run(self, nsteps):
        N.map_graph_run(self.ctx, self.U, self.dt, nsteps, self.sp)

    def flags(self):
        return N.map_status_flags(self.ctx, self.sp)

    def set_launch(self, mode, grid_step=0, grid_fill=0):
        N.map_set_launch(self.ctx, mode, grid_step, grid_fill)

    def autotune(self):
        """Pick the launch shapes (map_autotune) and return them (map_get_launch)."""
        N.map_autotune(self.ctx, self.U, self.sp)
        return N.map_get_launch(self.ctx)

    def launch_config(self) -> dict:
        return N.map_get_launch(self.ctx)

    def set_launch_config(self, **cfg):
        N.map_set_launch_config(self.ctx, cfg)

    # ---------------------------------------------------------------- regrid
    def estimate(self, criteria, filt=0.05, bias=0.6, ratio=2.0, xi=0.0):
        """Per-block regrid estimate (Sec. 4.5) in the caller's key order
        (float64 numpy); criteria as in native.make_estimator."""
        est = N.make_estimator(criteria, filt=filt, bias=bias, ratio=ratio, xi=xi)
        err = torch.zeros(self.nslots, dtype=torch.float64, device=self.device)
        torch.cuda.synchronize(self.device)
        N.map_estimate(self.ctx, self.U, est, err, self.sp)
        self.stream.synchronize()
        return err.cpu().numpy()[self.slot_of_key]

    def regrid_interval(self, c_r=1.0):
        """(simulated time, whole steps) until the next regrid per simulation,
        from the last dt records (map_regrid_interval, Sec. 4.5)."""
        self.stream.synchronize()
        return N.map_regrid_interval(self.ctx, self.dt.cpu().numpy(), c_r)

    def regrid_in_place(self, criteria, tau_refine, tau_coarsen, max_level, **est_kw):
        """One regrid that re-plans this simulation in place: estimate on
        device, tree edit on the host, a new context bound to the second pair
        of state and workspace buffers, the state moved onto it, and the two
        pairs swapped.  A pair that is too small for the new tree is replaced
        by one of twice the tree's size, so once the tree sizes settle the
        regrids allocate nothing.  The launch shapes carry over."""
        import dataclasses
        est = N.make_estimator(criteria, **est_kw)
        err = torch.zeros(self.nslots, dtype=torch.float64, device=self.device)
        torch.cuda.synchronize(self.device)
        N.map_estimate(self.ctx, self.U, est, err, self.sp)
        self.stream.synchronize()
        keys = N.map_regrid(self.ctx, err.cpu().numpy(), tau_refine, tau_coarsen, max_level)
        cfg = N.map_get_launch(self.ctx)
        new_ctx = N.map_init_blocks(self.params, self.wl.sims, keys)
        sizes, _ = N.map_query(new_ctx)
        u_need = sizes.nblocks * NV * sizes.tile_cells
        ws_need = sizes.workspace_bytes + 256
        if self._spare is None:
            self._spare = (torch.zeros(2 * u_need, dtype=self.dtype, device=self.device),
                           torch.zeros(2 * ws_need, dtype=torch.uint8, device=self.device))
        ubuf, wsbuf = self._spare
        if ubuf.numel() < u_need:  # a tree larger than this pair has held
            ubuf = torch.zeros(2 * u_need, dtype=self.dtype, device=self.device)
        if wsbuf.numel() < ws_need:
            wsbuf = torch.zeros(2 * ws_need, dtype=torch.uint8, device=self.device)
        old_ctx, old_U = self.ctx, self.U
        old_bufs = (self._ubuf, self._wsbuf)
        self.ctx = new_ctx
        self._plan(dataclasses.replace(self.wl, keys=keys))
        self._ubuf, self._wsbuf = ubuf, wsbuf
        self._bind()
        N.map_set_launch_config(self.ctx, cfg)
        N.map_remap(self.ctx, self.U, old_ctx, old_U, self.sp)  # synchronises the stream
        N.map_destroy(old_ctx)
        self._spare = old_bufs
        return keys

    def run_adaptive(self, nsteps, criteria, tau_refine, tau_coarsen, max_level, c_r=1.0,
                     graph=True, **est_kw):
        """nsteps cycles with the regrids of Sec. 4.5 inside the run: after
        every regrid (and at the start) the interval to the next one comes
        from the last dt records (map_regrid_interval; the whole steps of dt
        in c_r 2 n_g dx_min / alpha_g, the smallest over the simulations);
        the simulation is re-planned in place.  Returns [(cycle, nblocks)]
        of the regrids done."""
        run = self.graph_run if graph else self.advance
        done, log = 0, []
        self.stream.synchronize()
        if not bool(self.dt[:, 0].gt(0).all()):
            self.cfl()
        while done < nsteps:
            _, steps = self.regrid_interval(c_r)
            n = min(int(steps.min()), nsteps - done)
            run(n)
            done += n
            if done < nsteps:
                self.regrid_in_place(criteria, tau_refine, tau_coarsen, max_level, **est_kw)
                log.append((done, self.nslots))
        return log

    def regrid(self, criteria, tau_refine, tau_coarsen, max_level, **est_kw):
        """One regrid: estimate on device, the tree edit on the host, and the
        state moved onto the new tree on device.  Returns a new Simulation
        (this one is left unchanged)."""
        import dataclasses
        est = N.make_estimator(criteria, **est_kw)
        err = torch.zeros(self.nslots, dtype=torch.float64, device=self.device)
        torch.cuda.synchronize(self.device)
        N.map_estimate(self.ctx, self.U, est, err, self.sp)
        self.stream.synchronize()
        keys = N.map_regrid(self.ctx, err.cpu().numpy(), tau_refine, tau_coarsen, max_level)
        wl = dataclasses.replace(self.wl, keys=keys)
        new = Simulation(wl, device=self.device, stream=self.stream, precision=self.precision)
        N.map_remap(new.ctx, new.U, self.ctx, self.U, self.sp)
        return new

    def sync(self):
        self.stream.synchronize()
