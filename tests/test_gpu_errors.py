"""Failure handling of the C ABI on the GPU, forced from the host: each condition
returns its documented status and every kernel still completes normally."""
import numpy as np
import pytest

import scenes
from gpu_util import GpuRun

pytestmark = pytest.mark.gpu


def _blob(**kw):
    return scenes.random_blob(0, n_cells=(16, 16, 16), lo_cells=(5.0, 5.0, 5.0), ext_cells=(4, 4, 4), **kw)


def test_particle_outside_domain_reported():
    sc = _blob()
    sc.x[7] = np.array([0.1 / 16, 0.5, 0.5], np.float32)   # below a quarter cell
    run = GpuRun(sc)
    got = run.steps(1e-4, 1)
    assert got["status"] == run.ck.MPM_E_DOMAIN
    # the error is cleared by mpm_sync and the context stays usable
    assert run.ck.mpm_sync(run.ctx.h, run.stream) == run.ck.MPM_OK
    run.close()


def test_particle_leaving_domain_reported():
    sc = _blob(v_scale=0.0)
    sc.x[:] = np.array([0.5, 0.5, 15.6 / 16], np.float32) + 0 * sc.x
    sc.v[:, 2] = 50.0                                         # leaves through the top in one step
    run = GpuRun(sc)
    got = run.steps(1e-3, 1)
    assert got["status"] == run.ck.MPM_E_DOMAIN
    run.close()


def test_block_pool_capacity_reported():
    sc = _blob()
    run = GpuRun(sc, max_blocks=2)
    got = run.steps(1e-4, 1)
    assert got["status"] == run.ck.MPM_E_CAPACITY
    run.close()


def test_nonfinite_state_reported():
    sc = _blob()
    sc.F[3, 0, 0] = np.nan
    run = GpuRun(sc)
    got = run.steps(1e-4, 1)
    assert got["status"] == run.ck.MPM_E_NONFINITE
    run.close()


def test_stale_positions_reported():
    import torch
    sc = _blob()
    run = GpuRun(sc)
    ck = run.ck
    ck.check(ck.mpm_p2g(run.ctx.h, run.parts.c, 1e-4, run.stream))
    ck.check(ck.mpm_grid_update(run.ctx.h, 1e-4, run.stream))
    # move every particle by two blocks after its keys were taken
    cur = run.parts.current
    run.parts.state[cur, 0, :sc.n] += torch.tensor(8.0 / 16, device="cuda")
    ck.check(ck.mpm_g2p(run.ctx.h, run.parts.c, 1e-4, run.stream))
    assert ck.mpm_sync(run.ctx.h, run.stream) == ck.MPM_E_STALE
    run.close()


def test_host_side_argument_errors():
    sc = _blob()
    run = GpuRun(sc)
    ck = run.ck
    h = run.ctx.h
    p = run.parts.c
    saved = p.n
    p.n = sc.n + 1                  # n beyond capacity and stride
    assert ck.mpm_step(h, p, 1e-4, 1, run.stream) == ck.MPM_E_INVALID
    p.n = saved
    assert ck.mpm_step(h, p, float("nan"), 1, run.stream) == ck.MPM_E_INVALID
    assert ck.mpm_step(h, p, 1e-4, -1, run.stream) == ck.MPM_E_INVALID
    p.current = 2
    assert ck.mpm_p2g(h, p, 1e-4, run.stream) == ck.MPM_E_INVALID
    p.current = 0
    # g2p without a preceding p2g on this buffer
    assert ck.mpm_g2p(h, p, 1e-4, run.stream) == ck.MPM_E_INVALID
    assert ck.mpm_sync(h, run.stream) == ck.MPM_OK
    run.close()


def test_empty_particle_set():
    sc = _blob()
    run = GpuRun(sc)
    run.parts.c.n = 0
    assert run.ck.mpm_step(run.ctx.h, run.parts.c, 1e-4, 2, run.stream) == run.ck.MPM_OK
    assert run.ck.mpm_sync(run.ctx.h, run.stream) == run.ck.MPM_OK
    run.close()
