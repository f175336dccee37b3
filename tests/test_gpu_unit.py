"""The P2G fixed-point unit is step-global: a P2G takes it from a bound on its
contributions -- four times the largest contribution bound of the previous P2G, or,
for a state that did not come from this context's G2P, the exact bound the stress
pass forms -- and a particle above it (a state changed in place without
mpm_invalidate) is added with float atomics instead of through the tile.  Both paths
are compared with the FP64 checker here."""
import numpy as np
import pytest

import scenes
from gpu_util import GpuRun, log, nerr, oracle_state, oracle_step

pytestmark = pytest.mark.gpu


def _grids_match(tag, got, g, tol=1e-5):
    em, ep = nerr(got["m"], g["m"]), nerr(got["p"], g["p"])
    log("%s: grid m %.2e p %.2e" % (tag, em, ep))
    assert em <= tol and ep <= tol, tag


@pytest.mark.parametrize("scale", [1.0, 200.0])
def test_p2g_after_in_place_velocity_change(scale):
    """One step forms the bound; then the velocities of some particles are scaled in
    place (keys and stress stay valid) and the next P2G is compared with the checker.
    At scale 200 those particles exceed the bound and take the float-atomic path."""
    import torch
    sc = scenes.random_blob(7, model=scenes.FIXED_COROTATED, n_cells=(16, 16, 16), lo_cells=(5.0, 5.5, 4.5),
                            ext_cells=(5, 4, 6), F_scale=0.03, E=1e5, v_scale=0.5)
    run = GpuRun(sc)
    dt = 1e-4
    assert run.steps(dt, 1)["status"] == 0
    cur = run.parts.current
    pick = torch.arange(0, run.parts.n, 37, device="cuda")
    run.parts.state[cur, 3:6, pick] *= scale
    torch.cuda.synchronize()
    before = run.parts.read_by_id()
    got = run.phase_step(dt)
    assert got["status"] == 0
    st = oracle_state(before)
    _, g = oracle_step(sc, st, dt)
    _grids_match("in-place velocity x%g" % scale, got, g)
    for name in ("x", "v", "F"):
        e = nerr(got[name], getattr(st, name))
        log("  particles %s %.2e" % (name, e))
        assert e <= 1e-5, name
    run.close()
