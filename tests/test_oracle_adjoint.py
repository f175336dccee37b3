"""Pins of the oracle's reverse-mode step (the FP64 adjoint the differentiable
rollout is checked against): central finite differences of the oracle's own
forward step, which is pinned separately, in seeded random directions.

  * the fixed-corotated stress adjoint (polar-factor derivative, determinant,
    modulus) against differences of the stress;
  * one whole step: every input (x, v, B, F, log E) against differences of
    <random cotangents, step(state)>;
  * a short rollout's centre-of-mass loss against differences along random
    directions of the initial velocity and the log-modulus field.
A dropped term, a sign or a transposed operand in any product rule moves one of
these by far more than the tolerance."""
import numpy as np
import pytest

import oracle
import scenes


def _fc_material(E=5e4, nu=0.3, rho=1000.0, vol0=1e-6):
    return oracle.material(0, E, nu, rho, vol0)


@pytest.mark.parametrize("scale", [0.01, 0.3])
def test_fc_stress_adjoint_matches_differences(scale):
    rng = np.random.default_rng(7)
    m = _fc_material()
    checked = 0
    while checked < 4:
        F = np.eye(3) + scale * rng.standard_normal((3, 3))
        if np.linalg.det(F) <= 0.2:
            continue
        checked += 1
        logE = np.log(5e4) + 0.1 * rng.standard_normal()
        tb = rng.standard_normal((3, 3))
        dF = rng.standard_normal((3, 3))
        h = 1e-6
        fd = float((tb * (oracle.kirchhoff(m, F + h * dF, logE) - oracle.kirchhoff(m, F - h * dF, logE))).sum()
                   / (2 * h))
        fdE = float((tb * (oracle.kirchhoff(m, F, logE + h) - oracle.kirchhoff(m, F, logE - h))).sum() / (2 * h))
        Fb, lb = oracle.kirchhoff_vjp(m, F, logE, tb)
        an = float((Fb * dF).sum())
        assert abs(an - fd) <= 1e-7 * max(1.0, abs(fd)), (an, fd)
        assert abs(lb - fdE) <= 1e-7 * max(1.0, abs(fdE)), (lb, fdE)


def _tiny_scene(seed, F_scale=0.05, gravity=(0.3, -9.8, 0.1), bc_band=2, lo_cells=(4.3, 4.6, 4.1)):
    sc = scenes.random_blob(seed, n_cells=(12, 12, 12), lo_cells=lo_cells, ext_cells=(3, 2, 2),
                            model=scenes.FIXED_COROTATED, v_scale=0.5, B_scale=2.0, F_scale=F_scale,
                            gravity=gravity, bc_band=bc_band, dt=1e-4, E=5e4)
    rng = np.random.default_rng(seed + 100)
    logE = np.log(5e4) + 0.2 * rng.standard_normal(sc.n)
    st = oracle.State(sc.x, sc.v, sc.B, sc.F, sc.mat, logE)
    return sc, st


def _pairing(cfg, mats, st, dt, cot):
    s = st.copy()
    status, _, _ = oracle.step(cfg, mats, s, dt)
    assert status == 0
    return float((cot[0] * s.x).sum() + (cot[1] * s.v).sum() + (cot[2] * s.B).sum() + (cot[3] * s.F).sum())


@pytest.mark.parametrize("near_wall", [False, True])
@pytest.mark.parametrize("field", ["x", "v", "B", "F", "logE"])
def test_step_adjoint_matches_differences(field, near_wall):
    """near_wall puts the particles against the sticky band, so that some of their
    nodes are held at zero velocity."""
    sc, st = _tiny_scene(3, lo_cells=(2.1, 2.3, 4.1) if near_wall else (4.3, 4.6, 4.1))
    cfg, mats = oracle.scene_config(sc), oracle.scene_materials(sc)
    dt = 1e-4
    rng = np.random.default_rng(11)
    n = st.n
    cot = [rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), rng.standard_normal((n, 3, 3)) * 64,
           rng.standard_normal((n, 3, 3))]
    status, g = oracle.step_vjp(cfg, mats, st, dt, *cot)
    assert status == 0
    base = getattr(st, field)
    d = rng.standard_normal(base.shape)
    # relative step: positions move a small fraction of a cell, the rest by ~1e-6
    h = {"x": 1e-7 * sc.dx * 16, "v": 1e-6, "B": 1e-6 * sc.dx, "F": 1e-6, "logE": 1e-6}[field]
    sp, sm = st.copy(), st.copy()
    setattr(sp, field, base + h * d)
    setattr(sm, field, base - h * d)
    fd = (_pairing(cfg, mats, sp, dt, cot) - _pairing(cfg, mats, sm, dt, cot)) / (2 * h)
    an = float((g[field] * d).sum())
    assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-12), (field, an, fd)


@pytest.mark.parametrize("loss_name", ["com", "spread"])
def test_rollout_gradient_matches_differences(loss_name):
    """12 steps of a small elastic box (the differentiation workload's material and
    time step), gradient in v0 and log E along seeded random directions, for the
    centre-of-mass loss and for the spread about the centre of mass.  Internal
    stress conserves momentum, so the centre of mass of a body that touches no wall
    does not depend on its stiffness: there the log E gradient must vanish (to
    rounding), which the spread loss then checks is not an artefact."""
    sc = scenes.diff_box(scale=4)
    # a prestrained body, so that stress (and with it the modulus) moves the particles
    rng0 = np.random.default_rng(9)
    sc.F = (np.eye(3)[None] + 0.02 * rng0.standard_normal((sc.n, 3, 3))).astype(np.float32)
    cfg, mats = oracle.scene_config(sc), oracle.scene_materials(sc)
    st0 = oracle.State.from_scene(sc)
    loss = oracle.com_loss(scenes.diff_target(scale=4)) if loss_name == "com" else oracle.spread_loss
    nsteps = 12
    value, g = oracle.rollout_loss_grad(cfg, mats, st0, sc.dt, nsteps, loss)
    assert value > 0
    if loss_name == "com":
        gv = np.abs(g["v"]).max()
        assert np.abs(g["logE"]).max() <= 1e-10 * gv, (np.abs(g["logE"]).max(), gv)
    rng = np.random.default_rng(5)
    for k in range(6):
        field = "v" if (k % 2 == 0 or loss_name == "com") else "logE"
        base = getattr(st0, field)
        d = rng.standard_normal(base.shape)
        d /= np.linalg.norm(d)
        # the losses are smooth and small: a step of 1e-3 keeps the rounding of the
        # two losses (~1e-17) well below 1e-7 of the slope
        h = 1e-3
        sp, sm = st0.copy(), st0.copy()
        setattr(sp, field, base + h * d)
        setattr(sm, field, base - h * d)
        fd = (oracle.rollout_loss(cfg, mats, sp, sc.dt, nsteps, loss)
              - oracle.rollout_loss(cfg, mats, sm, sc.dt, nsteps, loss)) / (2 * h)
        an = float((g[field] * d).sum())
        assert abs(an - fd) <= 1e-6 * abs(fd), (field, an, fd)
