"""Parity of the FP32 HIP step with the FP64 checker, through the C ABI.

Each comparison is a normalised L-infinity error max|gpu - ref| / max|ref| per
field, bounded by 1e-5:
  * per phase from identical input: grid mass and momentum after mpm_p2g, grid
    velocity after mpm_grid_update, particle x, v, B, F after mpm_g2p;
  * over the first 10 steps of the elastic cube (plain, perturbed, and touching
    the sticky floor) and of a reduced sand column, with the checker running its
    own FP64 trajectory from the same initial state (grids compared every step);
  * the first ten steps of the full 4,194,304-particle sand column (particles
    every step, grids after steps 1, 5 and 10), with mpm_step's step sequence and
    the fused G2P2G step checked against the same FP64 trajectory after steps 5
    and 10.
"""
import numpy as np
import pytest

import scenes
from gpu_util import TOL, GpuRun, log, nerr, oracle_state, oracle_step

pytestmark = pytest.mark.gpu


def _cmp_particles(tag, got, st, dx, tol=TOL):
    """x, v, F against the FP64 reference (the contract), B for information and
    with a floor on its scale: B has units of velocity x length, and for a rigid
    translation the reference B is zero up to FP64 rounding, so it is normalised
    by max(|B_ref|, dx |v_ref|)."""
    errs = {name: nerr(got[name], getattr(st, name)) for name in ("x", "v", "F")}
    bscale = max(np.abs(st.B).max(), dx * np.abs(st.v).max())
    eB = np.abs(got["B"] - st.B).max() / bscale
    dF = nerr(got["F"] - np.eye(3), st.F - np.eye(3))
    log("%s particles %s B=%.2e (F-I: %.2e)" % (tag, " ".join("%s=%.2e" % kv for kv in errs.items()), eB, dF))
    for name, e in errs.items():
        assert e <= tol, "%s: %s error %.3e" % (tag, name, e)
    assert eB <= 10 * tol, "%s: B error %.3e" % (tag, eB)


def _cmp_grids(tag, got, g, tol=TOL):
    """Grid mass and momentum after P2G, and the momentum m v~ after the update
    (v~ itself is a ratio of two sums and loses relative precision on nearly
    empty nodes; its error is logged)."""
    em = nerr(got["m"], g["m"])
    ep = nerr(got["p"], g["p"])
    emv = nerr(got["m"][..., None].astype(np.float64) * got["vt"], g["m"][..., None] * g["v"])
    ev = nerr(got["vt"], g["v"])
    log("%s grid m=%.2e p=%.2e m*v~=%.2e (v~ %.2e)" % (tag, em, ep, emv, ev))
    assert em <= tol and ep <= tol and emv <= tol, tag


PHASE_CASES = {
    "fc_free": dict(seed=0, model=scenes.FIXED_COROTATED, n_cells=(16, 16, 16), lo_cells=(5.5, 6.25, 4.75),
                    ext_cells=(5, 4, 6), F_scale=0.05, E=1e5),
    "dp_free": dict(seed=1, model=scenes.DRUCKER_PRAGER, n_cells=(16, 16, 16), lo_cells=(4.0, 5.0, 6.0),
                    ext_cells=(6, 5, 4), F_scale=0.03, E=3.5e5),
    "fc_walls": dict(seed=2, model=scenes.FIXED_COROTATED, n_cells=(16, 16, 16), lo_cells=(1.25, 1.5, 2.0),
                     ext_cells=(13, 6, 12), gravity=(0.0, -9.8, 0.0), bc_band=2, F_scale=0.02),
    "dp_walls": dict(seed=3, model=scenes.DRUCKER_PRAGER, n_cells=(32, 16, 16), lo_cells=(1.5, 1.25, 3.0),
                     ext_cells=(29, 7, 10), gravity=(0.5, -9.8, 0.0), bc_band=2, F_scale=0.05, E=3.5e5),
    "fc_inverted": dict(seed=4, model=scenes.FIXED_COROTATED, n_cells=(16, 16, 16), lo_cells=(5.0, 5.0, 5.0),
                        ext_cells=(3, 3, 3), F_scale=0.6),
    # strains below the series threshold (|FF^T - I|_F <= 0.05): matrix-series constitutive path
    "fc_small_strain": dict(seed=5, model=scenes.FIXED_COROTATED, n_cells=(16, 16, 16), lo_cells=(4.5, 5.0, 5.5),
                            ext_cells=(6, 5, 4), F_scale=0.004, E=1e5),
    "dp_small_strain": dict(seed=6, model=scenes.DRUCKER_PRAGER, n_cells=(16, 16, 16), lo_cells=(5.0, 4.5, 4.0),
                            ext_cells=(5, 6, 5), F_scale=0.004, E=3.5e5),
}


@pytest.mark.parametrize("case", sorted(PHASE_CASES))
def test_phase_parity_one_step(case):
    sc = scenes.random_blob(**PHASE_CASES[case])
    dt = 1e-4
    run = GpuRun(sc)
    got = run.phase_step(dt)
    run.close()
    assert got["status"] == 0
    st = oracle_state(dict(x=sc.x, v=sc.v, B=sc.B, F=sc.F))
    _, g = oracle_step(sc, st, dt)
    _cmp_grids(case, got, g)
    _cmp_particles(case, got, st, sc.dx)


TRAJ = {
    "cube_elastic": (scenes.cube_elastic, 10),
    "cube_elastic_perturbed": (lambda: scenes.cube_elastic_perturbed(1), 10),
    "cube_elastic_floor": (lambda: scenes.cube_elastic_perturbed(1, floor_cells=2.5), 10),
    "sand_column_quarter": (lambda: scenes.sand_column(scale=4), 10),
}


@pytest.mark.parametrize("name", sorted(TRAJ))
def test_trajectory_ten_steps(name):
    builder, nsteps = TRAJ[name]
    sc = builder()
    run = GpuRun(sc)
    st = oracle_state(dict(x=sc.x, v=sc.v, B=sc.B, F=sc.F))
    for k in range(nsteps):
        got = run.phase_step(sc.dt)
        assert got["status"] == 0, "step %d status %d" % (k, got["status"])
        _, g = oracle_step(sc, st, sc.dt)
        _cmp_grids("%s step %d" % (name, k + 1), got, g)
        _cmp_particles("%s step %d" % (name, k + 1), got, st, sc.dx)
    run.close()


@pytest.mark.parametrize("name", ["cube_elastic_perturbed", "sand_column_quarter"])
def test_reseeded_step_parity(name):
    """Each step checked from the GPU's own state, so the bound covers the step
    alone and not the divergence of two trajectories."""
    sc = TRAJ[name][0]()
    run = GpuRun(sc)
    for k in range(5):
        before = run.parts.read_by_id()
        got = run.steps(sc.dt, 1)
        assert got["status"] == 0
        st = oracle_state(before)
        oracle_step(sc, st, sc.dt, grids=False)
        _cmp_particles("%s reseeded step %d" % (name, k + 1), got, st, sc.dx)
    run.close()


@pytest.mark.timeout(1200)
def test_full_sand_column_ten_steps():
    """The 4,194,304-particle sand column at full size: ten phase steps against the
    checker's own FP64 trajectory from the same initial state, particle x, v, F every
    step and grid mass, momentum and m v~ after steps 1, 5 and 10.  Beside them, from
    the same initial state, two mpm_step calls of five steps (inside a call every G2P
    but the last hands Q to the next P2G in place of B and the stress) and two fused
    G2P2G calls of five steps, compared with the same trajectory after steps 5 and 10."""
    sc = scenes.sand_column()
    assert sc.n == 4194304
    run = GpuRun(sc)
    seq = GpuRun(sc)
    fused = GpuRun(sc, fused=True)
    st = oracle_state(dict(x=sc.x, v=sc.v, B=sc.B, F=sc.F))
    for k in range(10):
        with_grids = k + 1 in (1, 5, 10)
        got = run.phase_step(sc.dt, want_grids=with_grids)
        assert got["status"] == 0, "step %d status %d" % (k + 1, got["status"])
        _, g = oracle_step(sc, st, sc.dt, grids=with_grids)
        if with_grids:
            _cmp_grids("sand_column full, step %d" % (k + 1), got, g)
            del g
        _cmp_particles("sand_column full, step %d" % (k + 1), got, st, sc.dx)
        if k + 1 in (5, 10):
            for tag, r in (("mpm_step", seq), ("fused", fused)):
                got = r.steps(sc.dt, 5)
                assert got["status"] == 0, "%s step %d status %d" % (tag, k + 1, got["status"])
                _cmp_particles("sand_column full, %s, step %d" % (tag, k + 1), got, st, sc.dx)
        del got
    run.close()
    seq.close()
    fused.close()


def test_mpm_step_equals_phase_calls():
    """mpm_step and the three phase calls run the same kernels: same ids in the
    same sorted order and the same state up to atomic summation order."""
    sc = scenes.cube_elastic_perturbed(1)
    a = GpuRun(sc)
    b = GpuRun(sc)
    for _ in range(3):
        a.phase_step(sc.dt, want_grids=False)
    got_b = b.steps(sc.dt, 3)
    got_a = a.parts.read()
    raw_b = b.parts.read()
    assert np.array_equal(got_a["id"], raw_b["id"])
    for name in ("x", "v", "F"):
        assert nerr(got_a[name], raw_b[name]) < 1e-6
    assert got_b["status"] == 0
    a.close()
    b.close()
