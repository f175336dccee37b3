"""The exact-gradient transfers on the GPU (MPM_TRANSFER_APIC, section 4.4, and
MPM_TRANSFER_PIC, section 4.3) against the oracle's same transfers: one step per
phase from identical input and ten-step trajectories against the oracle's own FP64
trajectory."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_util import TOL, GpuRun, log, nerr, oracle_state

pytestmark = pytest.mark.gpu

NAMES = {1: "apic", 2: "pic"}


def _ora_step(sc, st, dt, transfer):
    status, _, g = oracle.step(oracle.scene_config(sc, transfer), oracle.scene_materials(sc), st, dt, grids=True)
    assert status == 0
    return g


def _cmp(tag, got, st, g, transfer):
    errs = {k: nerr(got[k], getattr(st, k)) for k in ("x", "v", "F")}
    em = nerr(got["m"], g["m"])
    ep = nerr(got["p"], g["p"])
    emv = nerr(got["m"][..., None].astype(np.float64) * got["vt"], g["m"][..., None] * g["v"])
    log("%s %s: %s grid m=%.2e p=%.2e m*v~=%.2e" % (tag, NAMES[transfer], " ".join("%s=%.2e" % kv for kv in errs.items()),
                                                    em, ep, emv))
    assert em <= TOL and ep <= TOL and emv <= TOL, tag
    for k, e in errs.items():
        assert e <= TOL, (tag, k, e)
    if transfer == 2:
        assert np.abs(got["B"]).max() == 0.0
    else:
        # B has units of velocity x length; for a nearly rigid motion the reference B
        # is small, so its error is normalised by max(|B|, |v| / 32 cells) as in the
        # MLS parity tests
        bscale = max(np.abs(st.B).max(), np.abs(st.v).max() / 32.0)
        assert np.abs(got["B"] - st.B).max() <= 10 * TOL * bscale


CASES = {
    "fc_free": dict(seed=0, model=scenes.FIXED_COROTATED, n_cells=(16, 16, 16), lo_cells=(5.5, 6.25, 4.75),
                    ext_cells=(5, 4, 6), F_scale=0.05, E=1e5),
    "dp_walls": dict(seed=3, model=scenes.DRUCKER_PRAGER, n_cells=(32, 16, 16), lo_cells=(1.5, 1.25, 3.0),
                     ext_cells=(29, 7, 10), gravity=(0.5, -9.8, 0.0), bc_band=2, F_scale=0.05, E=3.5e5),
    "fc_walls": dict(seed=2, model=scenes.FIXED_COROTATED, n_cells=(16, 16, 16), lo_cells=(1.25, 1.5, 2.0),
                     ext_cells=(13, 6, 12), gravity=(0.0, -9.8, 0.0), bc_band=2, F_scale=0.02),
}


@pytest.mark.parametrize("transfer", [1, 2])
@pytest.mark.parametrize("case", sorted(CASES))
def test_transfer_phase_parity_one_step(case, transfer):
    sc = scenes.random_blob(**CASES[case])
    dt = 1e-4
    run = GpuRun(sc, transfer=transfer)
    got = run.phase_step(dt)
    run.close()
    assert got["status"] == 0
    st = oracle_state(dict(x=sc.x, v=sc.v, B=sc.B, F=sc.F))
    g = _ora_step(sc, st, dt, transfer)
    _cmp(case, got, st, g, transfer)


@pytest.mark.parametrize("transfer", [1, 2])
def test_transfer_trajectory_ten_steps(transfer):
    sc = scenes.cube_elastic_perturbed(1, floor_cells=2.5)
    run = GpuRun(sc, transfer=transfer)
    st = oracle_state(dict(x=sc.x, v=sc.v, B=sc.B, F=sc.F))
    for k in range(10):
        got = run.phase_step(sc.dt)
        assert got["status"] == 0
        g = _ora_step(sc, st, sc.dt, transfer)
        _cmp("cube on the floor, step %d" % (k + 1), got, st, g, transfer)
    run.close()


def test_transfer_flags_validated():
    from paper_2412_10399_amd import ckmpm
    sc = scenes.random_blob(1)
    for kw in (dict(transfer=1, fused=True), dict(transfer=2, quadratic=True)):
        s, h = ckmpm.mpm_create(ckmpm.scene_config(sc, **kw), ckmpm.scene_materials(sc))
        assert s == ckmpm.MPM_E_INVALID and not h.value
