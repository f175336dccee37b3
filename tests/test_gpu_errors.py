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


def _dense_block_scene(n, seed=0):
    """n particles inside the single block of G- cells 4..7 per axis of a 16^3 grid;
    the G- cell is floor(X + 1/4), so the block spans X in [3.75, 7.75)."""
    rng = np.random.default_rng(seed)
    sc = _blob()
    dx = sc.dx
    x = ((3.75 + 4.0 * rng.random((n, 3))) * dx).astype(np.float32)
    x = np.clip(x, np.float32(3.75 * dx), np.nextafter(np.float32(7.75 * dx), np.float32(0)))
    sc.x = x
    sc.v = (0.1 * rng.standard_normal((n, 3))).astype(np.float32)
    sc.B = np.zeros((n, 3, 3), np.float32)
    sc.F = np.tile(np.eye(3, dtype=np.float32), (n, 1, 1))
    sc.mat = np.zeros(n, np.uint8)
    return sc


def test_block_at_particle_capacity_matches_checker():
    import oracle
    from gpu_util import nerr, oracle_state, oracle_step
    sc = _dense_block_scene(2048)
    run = GpuRun(sc)
    got = run.steps(1e-4, 1)
    assert got["status"] == run.ck.MPM_OK
    st = oracle_state(dict(x=sc.x, v=sc.v, B=sc.B, F=sc.F))
    oracle_step(sc, st, 1e-4, grids=False)
    for name in ("x", "v", "F"):
        assert nerr(got[name], getattr(st, name)) < 1e-5
    s, stats = run.ck.mpm_get_stats(run.ctx.h, run.stream)
    assert s == 0 and stats.max_block_particles == 2048 and stats.n_particle_blocks == 1
    run.close()
    del oracle


def test_block_over_particle_capacity_reported():
    sc = _dense_block_scene(2049)
    run = GpuRun(sc)
    got = run.steps(1e-4, 1)
    assert got["status"] == run.ck.MPM_E_CAPACITY
    run.close()
