"""Pins of the oracle's constitutive models (fixed corotated, Drucker-Prager
return mapping) and its 3x3 SVD against LAPACK, closed forms and the energy
they derive from."""
import math

import numpy as np
import pytest

FC, DP = 0, 1


def _mat(ora, model, E=1e4, nu=0.3):
    return ora.material(model, E, nu, 1000.0, 1.0, 30.0)


def _lame(E, nu):
    return E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))


def _special_matrices():
    rng = np.random.default_rng(0)
    out = [np.eye(3), np.diag([2.0, 2.0, 1.0]), np.diag([1.0, 1.0, -1.0]), np.diag([3.0, 0.0, 0.0]),
           np.zeros((3, 3)), np.outer([1, 2, 3], [0.5, -1, 2.0]), np.diag([1.0, 1 + 1e-9, 1 - 1e-9])]
    for _ in range(40):
        out.append(rng.standard_normal((3, 3)))
        out.append(np.eye(3) + 1e-3 * rng.standard_normal((3, 3)))
    return out


def test_svd_against_lapack(ora):
    for F in _special_matrices():
        U, S, V = ora.svd3(F)
        ref = np.linalg.svd(F, compute_uv=False)
        assert np.abs(np.abs(S) - ref).max() <= 1e-13 * max(1.0, ref.max())
        assert np.all(np.diff(np.abs(S)) <= 1e-15)
        assert np.abs(U @ np.diag(S) @ V.T - F).max() <= 1e-13 * max(1.0, np.abs(F).max())
        assert np.abs(U.T @ U - np.eye(3)).max() < 1e-13 and np.abs(V.T @ V - np.eye(3)).max() < 1e-13
        assert np.linalg.det(U) == pytest.approx(1.0, abs=1e-12)
        assert np.linalg.det(V) == pytest.approx(1.0, abs=1e-12)
        assert np.all(S[:2] >= 0)
        assert np.sign(S[2]) == np.sign(np.linalg.det(F)) or abs(S[2]) < 1e-12


def _rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


@pytest.mark.parametrize("model", [FC, DP])
def test_rotations_are_stress_free(ora, model):
    rng = np.random.default_rng(1)
    m = _mat(ora, model)
    for _ in range(20):
        R = _rotation(rng)
        assert np.abs(ora.kirchhoff(m, R)).max() < 1e-10


def test_fixed_corotated_hydrostatic_closed_form(ora):
    E, nu = 1e4, 0.3
    mu, lam = _lame(E, nu)
    m = _mat(ora, FC, E, nu)
    for s in (0.5, 0.9, 1.0, 1.1, 2.0):
        tau = ora.kirchhoff(m, s * np.eye(3))
        expect = 2 * mu * (s - 1) * s + lam * (s ** 3 - 1) * s ** 3
        assert np.abs(tau - expect * np.eye(3)).max() <= 1e-12 * max(1.0, abs(expect))


def test_drucker_prager_hydrostatic_closed_form(ora):
    E, nu = 3.5e5, 0.3
    mu, lam = _lame(E, nu)
    m = _mat(ora, DP, E, nu)
    for s in (0.5, 0.9, 1.0, 1.1):
        tau = ora.kirchhoff(m, s * np.eye(3))
        expect = (2 * mu + 3 * lam) * math.log(s)
        assert np.abs(tau - expect * np.eye(3)).max() <= 1e-9 * max(1.0, abs(expect))


@pytest.mark.parametrize("model", [FC, DP])
def test_kirchhoff_is_energy_derivative(ora, model):
    """tau = P F^T with P = d psi / d F, checked by central differences of the energy."""
    rng = np.random.default_rng(2)
    m = _mat(ora, model, E=2e4, nu=0.35)
    for _ in range(12):
        F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
        if np.linalg.det(F) <= 0.2:
            continue
        P = np.zeros((3, 3))
        h = 1e-6
        for i in range(3):
            for j in range(3):
                e = np.zeros((3, 3))
                e[i, j] = h
                P[i, j] = (ora.energy_density(m, F + e) - ora.energy_density(m, F - e)) / (2 * h)
        tau = ora.kirchhoff(m, F)
        assert np.abs(tau - tau.T).max() <= 1e-10 * np.abs(tau).max()
        assert np.abs(tau - P @ F.T).max() <= 1e-6 * np.abs(tau).max()


def test_per_particle_log_modulus(ora):
    m = _mat(ora, FC, E=5e4)
    F = np.eye(3) + 0.05 * np.random.default_rng(3).standard_normal((3, 3))
    assert np.abs(ora.kirchhoff(m, F, logE=math.log(5e4)) - ora.kirchhoff(m, F)).max() < 1e-9
    assert np.abs(ora.kirchhoff(m, F, logE=math.log(1e5)) - 2 * ora.kirchhoff(m, F)).max() < 1e-9


def _cone_terms(E, nu, phi, F):
    mu, lam = _lame(E, nu)
    s = np.linalg.svd(F, compute_uv=False)
    eps = np.log(s)
    tr = eps.sum()
    dev = eps - tr / 3
    sphi = math.sin(math.radians(phi))
    alpha = math.sqrt(2 / 3) * 2 * sphi / (3 - sphi)
    return np.linalg.norm(dev), tr, (3 * lam + 2 * mu) / (2 * mu) * tr * alpha


def test_drucker_prager_return_mapping(ora):
    E, nu, phi = 3.5e5, 0.3, 30.0
    m = _mat(ora, DP, E, nu)
    rng = np.random.default_rng(4)
    n_inside = n_tip = n_proj = 0
    for _ in range(300):
        R1, R2 = _rotation(rng), _rotation(rng)
        sig = np.exp(0.05 * rng.standard_normal(3))
        F = R1 @ np.diag(sig) @ R2
        dn, tr, c = _cone_terms(E, nu, phi, F)
        G = ora.dp_return_map(m, F)
        if tr > 0:
            n_tip += 1
            assert np.abs(G @ G.T - np.eye(3)).max() < 1e-12       # stress-free: a pure rotation
            assert np.abs(G - R1 @ R2).max() < 1e-12
        elif dn + c <= 0:
            n_inside += 1
            assert np.abs(G - F).max() == 0.0
        else:
            n_proj += 1
            dn2, tr2, c2 = _cone_terms(E, nu, phi, G)
            assert tr2 == pytest.approx(tr, abs=1e-13)             # volume kept
            assert dn2 + c2 == pytest.approx(0.0, abs=1e-12)       # on the yield surface
            # same singular vectors: G F^-1 is symmetric in the left frame
            assert np.abs(ora.dp_return_map(m, G) - G).max() < 1e-12   # idempotent
    assert n_inside > 10 and n_tip > 10 and n_proj > 10
    # alpha at 30 degrees, as stated for the sand workloads
    sphi = math.sin(math.radians(30.0))
    assert math.sqrt(2 / 3) * 2 * sphi / (3 - sphi) == pytest.approx(0.32660, abs=1e-5)
