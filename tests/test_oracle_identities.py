"""Pins of the oracle's dual-grid stencil and moment matrix (paper section 4.2,
section 4.4) against identities the paper states and closed forms derived here
from the kernel alone."""
import math

import numpy as np
import pytest


def _cfg(ora, dx=1.0):
    return ora.config((8, 8, 8), dx, origin=(0.1, -0.2, 0.3))


def _random_positions(n, seed, dx=1.0, origin=(0.1, -0.2, 0.3)):
    rng = np.random.default_rng(seed)
    return np.asarray(origin) + dx * (1.0 + 6.0 * rng.random((n, 3)))


def test_partition_of_unity_per_grid(ora):
    # eq. interpolation-kernel-sum-to-1 holds on each grid separately
    cfg = _cfg(ora)
    for xp in _random_positions(200, 0):
        _, w, _ = ora.stencil(cfg, xp)
        assert abs(w[0].sum() - 1) < 1e-14 and abs(w[1].sum() - 1) < 1e-14
        assert np.all(w >= 0)


def test_dual_grid_reconstructs_position(ora):
    # eq. new-reconstruction-of-position: 1/2 sum_k sum_i x_i w = x_p
    dx = 0.0625
    cfg = _cfg(ora, dx)
    for xp in _random_positions(200, 1, dx):
        nodes, w, d = ora.stencil(cfg, xp)
        xi = xp[None, None, :] + d
        rec = 0.5 * np.einsum("go,goa->a", w, xi)
        assert np.abs(rec - xp).max() < 1e-14
        # the paper's reason for the second grid: a single grid misses x_p by s/(2 pi)-sized terms
        single = np.einsum("o,oa->a", w[1], xi[1])
        assert np.abs(single - xp).max() > 1e-6 * dx or np.abs(d[1] / dx - np.round(d[1] / dx)).max() < 1e-9


def _closed_form_D(X):
    """Moment matrix in cell units from the per-axis moments of the kernel: on grid
    k the first moment of the two weights is -s_k and the second is
    xi(1 - xi) - s_k(1 - 2 xi), with s = sin(2 pi xi)/(2 pi); the G- fractional
    coordinate is the G+ one shifted by a half cell, so s_- = -s_+."""
    xi_p = np.mod(X - 0.25, 1.0)
    xi_m = np.mod(X + 0.25, 1.0)
    s_p = np.sin(2 * math.pi * xi_p) / (2 * math.pi)
    s_m = np.sin(2 * math.pi * xi_m) / (2 * math.pi)
    m1 = [-s_m, -s_p]
    m2 = [xi_m * (1 - xi_m) - s_m * (1 - 2 * xi_m), xi_p * (1 - xi_p) - s_p * (1 - 2 * xi_p)]
    D = np.zeros((3, 3))
    for g in range(2):
        D += 0.5 * (np.outer(m1[g], m1[g]) + np.diag(m2[g] - m1[g] ** 2))
    return D


def test_moment_matrix_closed_form(ora):
    cfg = ora.config((8, 8, 8), 1.0)
    for X in _random_positions(300, 2, 1.0, (0, 0, 0)):
        D = ora.moment_matrix(cfg, X)
        assert np.abs(D - _closed_form_D(X)).max() < 1e-15
        # the dual grids cancel the first moments: off-diagonals are s_a s_b
        s = np.sin(2 * math.pi * np.mod(X - 0.25, 1.0)) / (2 * math.pi)
        off = np.outer(s, s)
        for a in range(3):
            for b in range(3):
                if a != b:
                    assert abs(D[a, b] - off[a, b]) < 1e-15


def test_moment_matrix_scales_with_dx_and_eigen_bounds(ora):
    # eigenvalues of D/dx^2 lie in [3/16 - 1/(4 pi) - 1/(4 pi^2), 3/16 - 1/(4 pi) + 1/(2 pi^2)],
    # reached for xi on all three axes equal (the extremes of d - s^2 and d + 2 s^2)
    lo = 3 / 16 - 1 / (4 * math.pi) - 1 / (4 * math.pi ** 2)
    hi = 3 / 16 - 1 / (4 * math.pi) + 1 / (2 * math.pi ** 2)
    assert lo == pytest.approx(0.082592, abs=1e-6) and hi == pytest.approx(0.158583, abs=1e-6)
    dx = 0.125
    cfg = ora.config((8, 8, 8), dx)
    emin, emax = 1e9, -1e9
    for X in list(_random_positions(300, 3, 1.0, (0, 0, 0))) + [np.full(3, 2 + t) for t in np.linspace(0, 1, 401)]:
        ev = np.linalg.eigvalsh(ora.moment_matrix(cfg, X * dx)) / dx ** 2
        emin, emax = min(emin, ev.min()), max(emax, ev.max())
    assert emin >= lo - 1e-14 and emax <= hi + 1e-14
    assert emin == pytest.approx(lo, abs=1e-6) and emax == pytest.approx(hi, abs=1e-6)


@pytest.mark.parametrize("k", [-1, 1])
def test_moment_matrix_at_a_node(ora, k):
    # at a node of either grid the particle sits half a cell from the other grid's nodes:
    # D = dx^2/8 I, while the same particle's single-grid moment matrix is singular
    dx = 0.5
    cfg = ora.config((8, 8, 8), dx)
    X = np.array([3.0, 4.0, 5.0]) + k / 4.0
    D = ora.moment_matrix(cfg, X * dx)
    assert np.abs(D - dx * dx / 8 * np.eye(3)).max() < 1e-15
    nodes, w, d = ora.stencil(cfg, X * dx)
    g = 0 if k == -1 else 1
    Dsingle = np.einsum("o,oa,ob->ab", w[g], d[g], d[g])
    assert np.abs(Dsingle).max() < 1e-15
