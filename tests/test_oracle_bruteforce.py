"""The C++ oracle against the definition-level numpy brute force (all nodes of
both grids, LAPACK SVD) on tiny scenes: particles, grid mass, grid momentum and
grid velocity after one step agree to 1e-13 relative."""
import numpy as np
import pytest

import scenes
from oracle import bruteforce as bf


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = [
    dict(seed=0, model=scenes.FIXED_COROTATED),
    dict(seed=1, model=scenes.DRUCKER_PRAGER, F_scale=0.1),
    dict(seed=2, model=scenes.FIXED_COROTATED, gravity=(0.0, -9.8, 0.0), bc_band=3, lo_cells=(1.5, 1.5, 1.5)),
    dict(seed=3, model=scenes.DRUCKER_PRAGER, gravity=(1.0, -9.8, 0.5), bc_band=2, lo_cells=(1.25, 2.5, 3.0),
         E=3.5e5),
    dict(seed=4, model=scenes.FIXED_COROTATED, ext_cells=(1, 1, 1), lo_cells=(3.0, 3.0, 3.0)),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("transfer", [0, 1, 2])
def test_oracle_matches_bruteforce(ora, case, transfer):
    sc = scenes.random_blob(**case)
    st = ora.State.from_scene(sc)
    x0, v0, B0, F0 = st.x.copy(), st.v.copy(), st.B.copy(), st.F.copy()
    dt = 1e-3
    status, diag, g = ora.step(ora.scene_config(sc, transfer), ora.scene_materials(sc), st, dt, grids=True)
    assert status == 0
    r = bf.step(sc, x0, v0, B0, F0, dt, transfer=("mls", "apic", "pic")[transfer])
    assert _rel(st.x, r["x"]) < 1e-13
    assert _rel(st.v, r["v"]) < 1e-13
    assert _rel(st.B, r["B"]) < 1e-13
    assert _rel(st.F, r["F"]) < 1e-13
    assert _rel(g["m"].reshape(2, -1), r["m"]) < 1e-13
    assert _rel(g["p"].reshape(2, -1, 3), r["p"]) < 1e-13
    assert _rel(g["v"].reshape(2, -1, 3), r["vt"]) < 1e-13


def test_paper_linear_momentum_scalar(ora):
    """Section 6.1: 33,552 unit-mass particles at 0.05 (1,1,1) m/s carry a momentum of
    norm about 2905.69 kg m/s; the oracle's particle momentum diagnostic must agree.
    The particles are placed at random inside a sphere-sized box (dx = 1/256)."""
    import os
    golden = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_scalars.txt")):
        if line.strip() and not line.startswith("#"):
            k, v, tol = line.split()
            golden[k] = (float(v), float(tol))
    n = int(golden["sphere_particles"][0])
    vv = golden["sphere_speed_component"][0]
    rng = np.random.default_rng(0)
    x = 0.5 + 0.01 * rng.random((n, 3))
    cfg = ora.config((16, 16, 16), 1.0 / 256, origin=(0.47, 0.47, 0.47))
    mats = (ora.OraMaterial * 1)(ora.material(0, 1e6, 0.4, 1.0, 1.0))
    st = ora.State(x, np.full((n, 3), vv), np.zeros((n, 3, 3)), np.tile(np.eye(3), (n, 1, 1)))
    status, diag, _ = ora.step(cfg, mats, st, 0.0)
    assert status == 0
    norm = np.linalg.norm(diag[1:4])
    ref, tol = golden["sphere_momentum_norm"]
    assert norm == pytest.approx(ref, rel=tol)
    rate, rtol = golden["linear_error_rate"]
    assert 0.0309 / norm == pytest.approx(rate, rel=rtol)
