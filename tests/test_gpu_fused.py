"""The fused step (each step's G2P and the next step's P2G in one kernel, section
3.2's G2P2G structure), selected with MPM_FLAG_FUSED_G2P2G: the same trajectory as
the phase calls and as the FP64 checker, conservation, and the report of a particle
that moves further than the fused kernel's reach.  The full-size sand column's ten
fused steps are checked with the phase steps, against one FP64 trajectory
(test_gpu_parity.py)."""
import dataclasses

import numpy as np
import pytest

import scenes
from gpu_util import TOL, GpuRun, log, nerr, oracle_state, oracle_step

pytestmark = pytest.mark.gpu

TRAJ = {
    "cube_elastic_perturbed": lambda: scenes.cube_elastic_perturbed(1),
    "cube_elastic_floor": lambda: scenes.cube_elastic_perturbed(1, floor_cells=2.5),
    "sand_column_quarter": lambda: scenes.sand_column(scale=4),
}


@pytest.mark.parametrize("name", sorted(TRAJ))
def test_fused_trajectory_matches_checker(name):
    """Ten steps in one call (nine fused kernels) against the checker's own FP64
    trajectory: particles, and the last step's grid mass and momentum m v~."""
    sc = TRAJ[name]()
    nsteps = 10
    run = GpuRun(sc, fused=True)
    got = run.steps(sc.dt, nsteps)
    assert got["status"] == 0
    m, vt = run.grids()
    st = oracle_state(dict(x=sc.x, v=sc.v, B=sc.B, F=sc.F))
    for _ in range(nsteps):
        _, g = oracle_step(sc, st, sc.dt)
    errs = {k: nerr(got[k], getattr(st, k)) for k in ("x", "v", "F")}
    em = nerr(m, g["m"])
    emv = nerr(m[..., None].astype(np.float64) * vt, g["m"][..., None] * g["v"])
    log("%s fused, %d steps: %s grid m=%.2e m*v~=%.2e" % (name, nsteps, " ".join("%s=%.2e" % kv for kv in errs.items()),
                                                          em, emv))
    for k, e in errs.items():
        assert e <= TOL, (k, e)
    assert em <= TOL and emv <= TOL
    run.close()


@pytest.mark.parametrize("nsteps", [1, 2, 6])
def test_fused_equals_unfused(nsteps):
    """Same particles in the same sorted order, same values up to summation order."""
    sc = scenes.sand_column(scale=4)
    a = GpuRun(sc, fused=True)
    b = GpuRun(sc, fused=False)
    da = a.steps(sc.dt, nsteps)
    db = b.steps(sc.dt, nsteps)
    assert da["status"] == 0 and db["status"] == 0
    ra, rb = a.parts.read(), b.parts.read()
    assert np.array_equal(ra["id"], rb["id"])
    for k in ("x", "v", "B", "F"):
        assert nerr(da[k], db[k]) < 1e-6, k
    ma, va = a.grids()
    mb, vb = b.grids()
    # v~ = p / m loses relative precision on nearly empty nodes (float atomics add the
    # block sums in a different order); compare the momentum m v~ as the parity tests do
    assert nerr(ma, mb) < 1e-6
    assert nerr(ma[..., None].astype(np.float64) * va, mb[..., None].astype(np.float64) * vb) < 1e-5
    # a following unfused phase step continues from the fused state
    pa = a.phase_step(sc.dt, want_grids=False)
    pb = b.phase_step(sc.dt, want_grids=False)
    assert pa["status"] == 0 and pb["status"] == 0
    for k in ("x", "v", "F"):
        assert nerr(pa[k], pb[k]) < 1e-6, k
    a.close()
    b.close()


@pytest.mark.parametrize("model", [scenes.FIXED_COROTATED, scenes.DRUCKER_PRAGER])
def test_fused_momentum_conserved(model):
    from test_gpu_invariants import _momenta
    sc = scenes.random_blob(11, model=model, n_cells=(32, 32, 32), lo_cells=(8, 9, 10), ext_cells=(12, 10, 9),
                            v_scale=1.0, B_scale=2.0, F_scale=0.05, E=1e5)
    run = GpuRun(sc, fused=True)
    P0, L0 = _momenta(dict(x=sc.x, v=sc.v, B=sc.B), sc)
    got = run.steps(1e-4, 20)
    assert got["status"] == 0
    P1, L1 = _momenta(got, sc)
    eP = np.abs(P1 - P0).max() / np.abs(P0).max()
    eL = np.abs(L1 - L0).max() / np.abs(L0).max()
    log("fused conservation over 20 steps: P %.2e  L %.2e" % (eP, eL))
    assert eP < 1e-5 and eL < 1e-5
    run.close()


def test_fused_reports_particle_beyond_reach():
    """One particle moving nine cells per step: the phase calls follow it, the fused
    step reports MPM_E_CFL (its grid only covers the blocks next to the particle's
    previous block)."""
    sc = scenes.random_blob(21, n_cells=(32, 32, 32), lo_cells=(6.0, 12.0, 12.0), ext_cells=(1, 1, 1), v_scale=0.0,
                            B_scale=0.0, F_scale=0.0)
    dt = 1e-4
    sc = dataclasses.replace(sc, x=sc.x[:1].copy(), v=np.array([[9.0 * sc.dx / dt, 0.0, 0.0]], np.float32),
                             B=sc.B[:1].copy(), F=sc.F[:1].copy(), mat=sc.mat[:1].copy())
    plain = GpuRun(sc, fused=False)
    got = plain.steps(dt, 2)
    assert got["status"] == 0
    assert abs(float(got["x"][0, 0]) - (float(sc.x[0, 0]) + 18.0 * sc.dx)) < 1e-5
    plain.close()
    run = GpuRun(sc, fused=True)
    assert run.steps(dt, 2)["status"] == run.ck.MPM_E_CFL
    run.close()
