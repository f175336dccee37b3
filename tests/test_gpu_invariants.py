"""Properties of the GPU step that hold at any size: momentum conservation (no
gravity, no walls), exact reproduction of affine velocity fields, determinism of
the sort and of the particle order, and conservation of particle ids."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_util import GpuRun, log, nerr

pytestmark = pytest.mark.gpu


def _momenta(d, sc):
    m = sc.materials[0].rho * sc.materials[0].vol0
    x = d["x"].astype(np.float64)
    v = d["v"].astype(np.float64)
    B = d["B"].astype(np.float64)
    P = m * v.sum(axis=0)
    L = m * np.cross(x, v).sum(axis=0)
    L += m * np.array([(B[:, 2, 1] - B[:, 1, 2]).sum(), (B[:, 0, 2] - B[:, 2, 0]).sum(), (B[:, 1, 0] - B[:, 0, 1]).sum()])
    return P, L


@pytest.mark.parametrize("model", [scenes.FIXED_COROTATED, scenes.DRUCKER_PRAGER])
def test_momentum_conserved_over_steps(model):
    sc = scenes.random_blob(11, model=model, n_cells=(32, 32, 32), lo_cells=(8, 9, 10), ext_cells=(12, 10, 9),
                            v_scale=1.0, B_scale=2.0, F_scale=0.05, E=1e5)
    run = GpuRun(sc)
    P0, L0 = _momenta(dict(x=sc.x, v=sc.v, B=sc.B), sc)
    got = run.steps(1e-4, 20)
    assert got["status"] == 0
    P1, L1 = _momenta(got, sc)
    eP = np.abs(P1 - P0).max() / np.abs(P0).max()
    eL = np.abs(L1 - L0).max() / np.abs(L0).max()
    log("GPU conservation over 20 steps: P %.2e  L %.2e" % (eP, eL))
    assert eP < 1e-5 and eL < 1e-5
    run.close()


def test_affine_field_reproduced():
    rng = np.random.default_rng(3)
    sc = scenes.random_blob(12, n_cells=(32, 32, 32), lo_cells=(8, 8, 8), ext_cells=(10, 10, 10), F_scale=0.0)
    a = rng.standard_normal(3)
    A = rng.standard_normal((3, 3))
    cfg = oracle.scene_config(sc)
    x = sc.x.astype(np.float64)
    D = np.stack([oracle.moment_matrix(cfg, xp) for xp in x])
    sc.v = (a[None, :] + x @ A.T).astype(np.float32)
    sc.B = np.einsum("ab,pbc->pac", A, D).astype(np.float32)
    run = GpuRun(sc)
    dt = 1e-4
    got = run.steps(dt, 1)
    assert got["status"] == 0
    vexp = a[None, :] + x @ A.T
    assert nerr(got["v"], vexp) < 2e-6
    assert np.abs(got["F"] - (np.eye(3) + dt * A)[None]).max() < 1e-6
    Bexp = np.einsum("ab,pbc->pac", A, D)
    eB = nerr(got["B"], Bexp)
    log("affine reproduction on the GPU: v %.2e  B %.2e" % (nerr(got["v"], vexp), eB))
    # FP32 bound on B (a reading of the precision, derived, not fitted).  Every P2G
    # contribution to node i is w m v(x_i) here (tau = 0, B = A D), rounded in FP32
    # (at most four roundings), summed exactly, converted back and divided by the
    # node mass: the node velocity carries an error of at most eta |v|, eta = 8 u
    # (u = 2^-24).  B = 1/2 sum_k sum_i w v~_i (x_i - x_p)^T weighs that error by the
    # first absolute moment of the weights, 2 xi (1 - xi) - s (1 - 2 xi) <= 1/2 cell
    # per axis, so |dB| <= eta max|v| dx / 2; the FP32 sums of G2P, taken on velocity
    # differences, add at most 16 u relative to B.
    u = 2.0 ** -24
    bound = 0.5 * 8 * u * np.abs(vexp).max() * sc.dx / np.abs(Bexp).max() + 16 * u
    log("affine reproduction: B error %.2e, FP32 bound %.2e" % (eB, bound))
    assert eB <= bound
    run.close()


def test_runs_are_deterministic_in_order_and_close_in_value():
    sc = scenes.sand_column(scale=4)
    a = GpuRun(sc)
    b = GpuRun(sc)
    da = a.steps(sc.dt, 5)
    db = b.steps(sc.dt, 5)
    ra, rb = a.parts.read(), b.parts.read()
    assert np.array_equal(ra["id"], rb["id"])                      # identical sorted order
    assert np.array_equal(np.sort(ra["id"]), np.arange(sc.n))      # every particle kept exactly once
    for name in ("x", "v", "F"):
        assert nerr(da[name], db[name]) < 1e-6                     # only atomic summation order differs
    a.close()
    b.close()
