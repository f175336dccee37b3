"""Pins of the oracle's transfers and grid update against what the paper proves
and what the mathematics forces:
  * conservation of linear and angular momentum through P2G, the grid update and
    G2P (supplement theorems 1.1, 2.1, 2.2), with the grid totals carrying the
    factor 1/2 over both grids;
  * exact reproduction of an affine velocity field by the APIC/MLS transfers;
  * the grid stress force equals minus the derivative of the elastic energy with
    respect to node motion (the force of section 4.3 as an energy gradient), which
    fixes its sign, the stress measure, the volume factor and D^-1;
  * gravity and sticky walls in the grid update.
"""
import numpy as np
import pytest

import scenes


def _run(ora, sc, dt, transfer=0, grids=False):
    st = ora.State.from_scene(sc)
    cfg = ora.scene_config(sc, transfer)
    status, diag, g = ora.step(cfg, ora.scene_materials(sc), st, dt, grids=grids)
    assert status == 0
    return st, diag, g


@pytest.mark.parametrize("model", [scenes.FIXED_COROTATED, scenes.DRUCKER_PRAGER])
@pytest.mark.parametrize("transfer", [0, 1])
@pytest.mark.parametrize("seed", [0, 7])
def test_momentum_conservation(ora, model, transfer, seed):
    sc = scenes.random_blob(seed, model=model, E=1e5, v_scale=1.0, B_scale=3.0, F_scale=0.1)
    _, d, _ = _run(ora, sc, 1e-3, transfer)
    P = [d[1:4], d[8:11], d[20:23], d[26:29]]   # particles, after P2G, after update, after G2P
    L = [d[4:7], d[11:14], d[23:26], d[29:32]]
    assert d[7] == pytest.approx(d[0], rel=1e-14)
    sP = np.abs(P[0]).max()
    sL = np.abs(L[0]).max()
    for p in P[1:]:
        assert np.abs(p - P[0]).max() <= 1e-12 * sP
    for l in L[1:]:
        assert np.abs(l - L[0]).max() <= 1e-12 * sL
    # internal forces cancel and exert no net torque (symmetric Kirchhoff stress)
    mv = sP
    assert np.abs(d[14:17]).max() * 1e-3 <= 1e-12 * mv
    assert np.abs(d[17:20]).max() * 1e-3 <= 1e-12 * sL


@pytest.mark.parametrize("model", [scenes.FIXED_COROTATED, scenes.DRUCKER_PRAGER])
def test_pic_linear_momentum_conservation(ora, model):
    """Section 4.3 with the supplement's first theorem: the PIC transfer conserves
    linear momentum through P2G, the grid update (no gravity, no walls) and G2P, and
    the particles come out with no affine matrix."""
    sc = scenes.random_blob(4, model=model, E=1e5, v_scale=1.0, B_scale=3.0, F_scale=0.1)
    st, d, _ = _run(ora, sc, 1e-3, 2)
    P0 = sc.materials[0].rho * sc.materials[0].vol0 * sc.v.astype(np.float64).sum(axis=0)
    s = np.abs(P0).max()
    for p in (d[8:11], d[20:23], d[26:29]):
        assert np.abs(p - P0).max() <= 1e-12 * s
    assert np.abs(st.B).max() == 0.0


def test_momentum_conservation_detects_missing_affine_term(ora):
    """Negative control: with B set but its contribution dropped from P2G the
    angular momentum identity fails, so the test above can see such a mistake."""
    sc = scenes.random_blob(3, model=scenes.FIXED_COROTATED, B_scale=3.0)
    _, d, _ = _run(ora, sc, 1e-3)
    sc0 = sc.copy()
    sc0.B[:] = 0
    _, d0, _ = _run(ora, sc0, 1e-3)
    # the particle angular momentum with B differs from the B-free grid value
    assert np.abs(d[4:7] - d0[11:14]).max() > 1e-6 * np.abs(d[4:7]).max()


@pytest.mark.parametrize("transfer", [0, 1])
def test_affine_field_reproduced_exactly(ora, transfer):
    """v_p = a + A x_p, B_p = A D_p, F = I (zero stress), no gravity or walls: one step
    gives v_p' = a + A x_p, C_p = B_p' D_p^-1 = A and F' = I + dt A."""
    rng = np.random.default_rng(5)
    sc = scenes.random_blob(9, model=scenes.FIXED_COROTATED, F_scale=0.0)
    a = rng.standard_normal(3)
    A = rng.standard_normal((3, 3))
    cfg = ora.scene_config(sc, transfer)
    x = sc.x.astype(np.float64)
    D = np.stack([ora.moment_matrix(cfg, xp) for xp in x])
    st = ora.State(x, a[None, :] + x @ A.T, np.einsum("ab,pbc->pac", A, D), np.tile(np.eye(3), (len(x), 1, 1)))
    dt = 1e-3
    status, _, _ = ora.step(cfg, ora.scene_materials(sc), st, dt)
    assert status == 0
    vexp = a[None, :] + x @ A.T
    assert np.abs(st.v - vexp).max() <= 1e-12 * np.abs(vexp).max()
    C = np.einsum("pab,pbc->pac", st.B, np.linalg.inv(D))
    assert np.abs(C - A[None]).max() <= 1e-12 * np.abs(A).max()
    assert np.abs(st.F - (np.eye(3) + dt * A)[None]).max() <= 1e-13
    assert np.abs(st.x - (x + dt * vexp)).max() <= 1e-14


@pytest.mark.parametrize("model", [scenes.FIXED_COROTATED, scenes.DRUCKER_PRAGER])
def test_force_is_energy_gradient(ora, model):
    """With the MLS gradient grad Phi_i = w D^-1 (x_i - x_p) a motion of the nodes
    x_i -> x_i + u_i deforms each particle as F -> (I + 1/2 sum_k sum_i u_i grad Phi_i^T) F.
    Each grid carries the full mass (1/2 sum_k m_i = sum_p m_p), so the per-grid force
    is f_i = -2 dE/du_i with E = sum_p V_p^0 psi(F_p).  The oracle's force, read off
    the grid momentum, must match central differences of the oracle's energy."""
    sc = scenes.random_blob(2, model=model, E=1e5, F_scale=0.08, n_cells=(8, 8, 8), ext_cells=(2, 2, 2))
    sc.gravity = (0.0, 0.0, 0.0)
    cfg = ora.scene_config(sc)
    mats = ora.scene_materials(sc)
    dt = 1e-3
    _, _, g1 = _run(ora, sc, dt, grids=True)
    _, _, g0 = _run(ora, sc, 0.0, grids=True)
    force = (g1["p"] - g0["p"]) / dt                    # [2, nz, ny, nx, 3]
    x = sc.x.astype(np.float64)
    F = sc.F.astype(np.float64)
    V0 = sc.materials[0].vol0
    sten = [ora.stencil(cfg, xp) for xp in x]
    Dinv = [np.linalg.inv(ora.moment_matrix(cfg, xp)) for xp in x]

    def energy(gsel, node, axis, u):
        E = 0.0
        for p in range(len(x)):
            nodes, w, d = sten[p]
            Fp = F[p].copy()
            for o in range(8):
                if tuple(nodes[gsel, o]) == node:
                    grad = w[gsel, o] * Dinv[p] @ d[gsel, o]
                    G = np.zeros((3, 3))
                    G[axis, :] = 0.5 * u * grad
                    Fp = (np.eye(3) + G) @ F[p]
            E += V0 * ora.energy_density(mats[0], Fp)
        return E

    rng = np.random.default_rng(4)
    checked = 0
    touched = [(gsel, tuple(int(v) for v in sten[p][0][gsel, o])) for p in range(len(x)) for gsel in range(2)
               for o in range(8)]
    for idx in rng.choice(len(touched), 6, replace=False):
        gsel, node = touched[idx]
        for axis in range(3):
            h = 1e-6
            dE = (energy(gsel, node, axis, h) - energy(gsel, node, axis, -h)) / (2 * h)
            f = force[gsel, node[2], node[1], node[0], axis]
            assert f == pytest.approx(-2.0 * dE, rel=2e-5, abs=1e-9 * abs(force).max())
            checked += 1
    assert checked == 18


def test_gravity_and_sticky_walls(ora):
    sc = scenes.random_blob(4, model=scenes.FIXED_COROTATED, F_scale=0.0, B_scale=0.0, v_scale=0.0,
                            lo_cells=(1.5, 1.5, 1.5), ext_cells=(5, 5, 5), gravity=(0.0, -9.8, 2.0), bc_band=2)
    dt = 1e-3
    _, _, g = _run(ora, sc, dt, grids=True)
    m, v = g["m"], g["v"]
    n = sc.n_cells[0]
    for gsel, k in ((0, -0.25), (1, 0.25)):
        coords = np.arange(n + 1) + k
        inner = (coords >= 2) & (coords <= n - 2)
        sel = (m[gsel] > 0) & inner[None, None, :] & inner[None, :, None] & inner[:, None, None]
        assert sel.sum() > 0
        # stress- and velocity-free particles: interior nodes move with gravity only
        assert np.abs(v[gsel][sel] - dt * np.array([0.0, -9.8, 2.0])).max() < 1e-13
        wall = (m[gsel] > 0) & ~(inner[None, None, :] & inner[None, :, None] & inner[:, None, None])
        assert wall.sum() > 0 and np.abs(v[gsel][wall]).max() == 0.0
        assert np.abs(v[gsel][m[gsel] == 0]).max() == 0.0
