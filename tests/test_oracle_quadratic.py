"""Pins of the oracle's quadratic B-spline step (the single-grid, 27-node kernel the
paper compares the compact kernel against): the B-spline's defining values and
moments, the C++ step against the definition-level numpy brute force (every node
of the grid), exact reproduction of an affine velocity field, and momentum
conservation through the transfers."""
import numpy as np
import pytest

import oracle
import scenes
from oracle import bruteforce as bf


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_bspline_values_and_moments():
    # values at the knots and the centre of the quadratic B-spline
    for r, want in ((0.0, 0.75), (0.5, 0.5), (-0.5, 0.5), (1.0, 0.125), (1.5, 0.0), (2.0, 0.0)):
        assert abs(oracle.Nq(r) - want) < 1e-15
    rng = np.random.default_rng(0)
    for xi in rng.uniform(0.5, 1.5, 50):
        r = np.arange(3) - xi   # the three nodes of a particle at xi from its base node
        w = np.array([oracle.Nq(v) for v in r])
        assert abs(w.sum() - 1.0) < 1e-15                 # partition of unity
        assert abs((w * r).sum()) < 1e-15                 # zero first moment
        assert abs((w * r * r).sum() - 0.25) < 1e-15      # second moment 1/4: D = dx^2/4 I


CASES = [
    dict(seed=0, model=scenes.FIXED_COROTATED, lo_cells=(2.5, 2.5, 2.5)),
    dict(seed=1, model=scenes.DRUCKER_PRAGER, F_scale=0.1, lo_cells=(2.5, 2.5, 2.5)),
    dict(seed=2, model=scenes.FIXED_COROTATED, gravity=(0.0, -9.8, 0.0), bc_band=2, lo_cells=(1.5, 1.5, 1.5)),
    dict(seed=3, model=scenes.DRUCKER_PRAGER, gravity=(1.0, -9.8, 0.5), bc_band=2, lo_cells=(1.25, 2.5, 3.0),
         E=3.5e5),
]


@pytest.mark.parametrize("case", CASES)
def test_quadratic_step_matches_bruteforce(case):
    sc = scenes.random_blob(**case)
    st = oracle.State.from_scene(sc)
    x0, v0, B0, F0 = st.x.copy(), st.v.copy(), st.B.copy(), st.F.copy()
    dt = 1e-3
    status, diag, g = oracle.step_quadratic(oracle.scene_config(sc), oracle.scene_materials(sc), st, dt, grids=True)
    assert status == 0
    r = bf.step_quadratic(sc, x0, v0, B0, F0, dt)
    for k in ("x", "v", "B", "F"):
        assert _rel(getattr(st, k), r[k]) < 1e-13, k
    assert _rel(g["m"].reshape(-1), r["m"]) < 1e-13
    assert _rel(g["p"].reshape(-1, 3), r["p"]) < 1e-13
    assert _rel(g["v"].reshape(-1, 3), r["vt"]) < 1e-13


def test_quadratic_affine_field_reproduced():
    rng = np.random.default_rng(4)
    sc = scenes.random_blob(12, n_cells=(16, 16, 16), lo_cells=(4, 4, 4), ext_cells=(6, 6, 6), F_scale=0.0)
    a = rng.standard_normal(3)
    A = rng.standard_normal((3, 3))
    x = sc.x.astype(np.float64)
    st = oracle.State(x, a[None, :] + x @ A.T, np.repeat((A * sc.dx ** 2 / 4)[None], sc.n, axis=0),
                      np.repeat(np.eye(3)[None], sc.n, axis=0))
    dt = 1e-4
    status, _, _ = oracle.step_quadratic(oracle.scene_config(sc), oracle.scene_materials(sc), st, dt)
    assert status == 0
    assert _rel(st.v, a[None, :] + x @ A.T) < 1e-12
    assert _rel(st.B, np.repeat((A * sc.dx ** 2 / 4)[None], sc.n, axis=0)) < 1e-12
    assert _rel(st.F, np.repeat((np.eye(3) + dt * A)[None], sc.n, axis=0)) < 1e-12


@pytest.mark.parametrize("model", [scenes.FIXED_COROTATED, scenes.DRUCKER_PRAGER])
def test_quadratic_momentum_conserved(model):
    sc = scenes.random_blob(5, model=model, n_cells=(16, 16, 16), lo_cells=(5, 5, 5), ext_cells=(4, 3, 5),
                            F_scale=0.05, E=1e5)
    st = oracle.State.from_scene(sc)
    status, diag, _ = oracle.step_quadratic(oracle.scene_config(sc), oracle.scene_materials(sc), st, 1e-4)
    assert status == 0
    P0, Pg, Pu, P1 = diag[1:4], diag[8:11], diag[20:23], diag[26:29]
    s = np.abs(P0).max()
    for P in (Pg, Pu, P1):
        assert np.abs(P - P0).max() <= 1e-12 * s
