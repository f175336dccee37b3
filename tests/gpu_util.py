"""Helpers shared by the GPU parity tests: run a scene through the HIP library
(C ABI via the ctypes binding) and through the FP64 checker, and compare."""
import sys

import numpy as np

import oracle
import scenes  # noqa: F401  (re-exported for tests)

TOL = 1e-5   # normalised L-infinity tolerance of the FP32 GPU step against the FP64 checker


def nerr(a, b):
    """max |a - b| / max |b| (0 when both are identically zero)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.abs(a - b).max() if a.size else 0.0
    s = np.abs(b).max() if b.size else 0.0
    if s == 0.0:
        return 0.0 if d == 0.0 else float("inf")
    return float(d / s)


def log(*args):
    print(*args, flush=True)
    sys.stdout.flush()


class GpuRun:
    """One scene resident on the GPU with its context and stream."""

    def __init__(self, sc, max_blocks=None, device="cuda:0", fused=False, quadratic=False, transfer=0,
                 deterministic=False):
        import torch
        from paper_2412_10399_amd import ckmpm
        self.torch = torch
        self.ck = ckmpm
        self.sc = sc
        self.ctx = ckmpm.Context(ckmpm.scene_config(sc, max_blocks=max_blocks, fused=fused, quadratic=quadratic,
                                                    transfer=transfer, deterministic=deterministic),
                                 ckmpm.scene_materials(sc))
        self.parts = ckmpm.particles_from_scene(sc, device)
        self.stream = torch.cuda.current_stream()
        nx, ny, nz = (c + 1 for c in sc.n_cells)
        self.dims = (2, nz, ny, nx)
        self._m = None
        self._vec = None

    def grids(self):
        torch = self.torch
        if self._m is None:
            n = int(np.prod(self.dims))
            self._m = torch.zeros(n, dtype=torch.float32, device="cuda")
            self._vec = torch.zeros(3 * n, dtype=torch.float32, device="cuda")
        self.ck.check(self.ck.mpm_grid_read(self.ctx.h, 0, self._m.data_ptr(), self._vec.data_ptr(), self.stream))
        torch.cuda.synchronize()
        return self._m.cpu().numpy().reshape(self.dims), self._vec.cpu().numpy().reshape(self.dims + (3,))

    def phase_step(self, dt, want_grids=True):
        ck = self.ck
        h = self.ctx.h
        out = {}
        ck.check(ck.mpm_p2g(h, self.parts.c, dt, self.stream), "mpm_p2g")
        if want_grids:
            out["m"], out["p"] = self.grids()
        ck.check(ck.mpm_grid_update(h, dt, self.stream), "mpm_grid_update")
        if want_grids:
            _, out["vt"] = self.grids()
        ck.check(ck.mpm_g2p(h, self.parts.c, dt, self.stream), "mpm_g2p")
        out["status"] = ck.mpm_sync(h, self.stream)
        out.update(self.parts.read_by_id())
        return out

    def steps(self, dt, n):
        ck = self.ck
        ck.check(ck.mpm_step(self.ctx.h, self.parts.c, dt, n, self.stream), "mpm_step")
        status = ck.mpm_sync(self.ctx.h, self.stream)
        d = self.parts.read_by_id()
        d["status"] = status
        return d

    def close(self):
        self.ctx.close()


def oracle_state(d):
    """FP64 checker state from a GPU read-back (by id)."""
    return oracle.State(d["x"], d["v"], d["B"], d["F"], d.get("mat"))


def oracle_step(sc, st, dt, grids=True):
    status, diag, g = oracle.step(oracle.scene_config(sc), oracle.scene_materials(sc), st, dt, grids=grids)
    assert status == 0
    return diag, g
