"""Pins of the oracle's compact kernel (paper section 4.1) against what the paper
and the mathematics fix: closed-form values, the seven kernel properties listed
in section 4.1, and exact C^2 (not C^3) smoothness.  Derivatives here are taken
by finite differences of the oracle's K1 itself, so they pin K1 and not a
second formula."""
import math
import os

import numpy as np
import pytest
from scipy import integrate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kernel_values.txt")


def test_closed_form_values(ora):
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 5
    for x, val in rows:
        assert ora.K1(float(x)) == pytest.approx(float(val), abs=1e-15)


def test_normalization(ora):
    val, err = integrate.quad(ora.K1, -1.0, 1.0, points=[0.0], epsabs=1e-13, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-13


def test_monotone_nonnegative_compact(ora):
    xs = np.linspace(0.0, 1.0, 4001)
    k = np.array([ora.K1(x) for x in xs])
    km = np.array([ora.K1(-x) for x in xs])
    assert np.all(np.diff(k[:-1]) < 0)           # strictly decreasing on [0, 1)
    assert np.array_equal(k, km)                 # even
    assert np.all(k >= 0)
    for x in (1.0, 1.0 + 1e-12, 1.3, 2.0, -1.0, -1.7):
        assert ora.K1(x) == 0.0


def test_partition_of_unity_1d(ora):
    # section 4.1 property 7 / eq. resemble-linear: K1(x) + K1(1 - x) = 1
    for x in np.linspace(0.0, 1.0, 1001):
        assert ora.K1(x) + ora.K1(1.0 - x) == pytest.approx(1.0, abs=1e-15)


def test_converges_to_dirac(ora):
    # section 4.1 property 5: K1(x/h)/h acts as a delta as h -> 0 on a smooth test function
    phi = lambda x: math.cos(3 * x) + x * x + 0.3 * x
    errs = []
    for h in (0.1, 0.01, 0.001):
        val, _ = integrate.quad(lambda x: ora.K1(x / h) / h * phi(x), -h, h, points=[0.0], epsabs=1e-13)
        errs.append(abs(val - phi(0.0)))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-5


def _d(f, x, h, order):
    if order == 1:
        return (f(x + h) - f(x - h)) / (2 * h)
    return (f(x + h) - 2 * f(x) + f(x - h)) / (h * h)


@pytest.mark.parametrize("x0", [0.0, 1.0, -1.0])
def test_c2_at_junctions(ora, x0):
    """One-sided first and second differences of K1 agree across x = 0 and x = +-1
    (C^2), while the third derivative jumps (the kernel is not C^3)."""
    f = ora.K1
    h = 1e-4
    # one-sided derivatives from polynomial fits of samples on each side
    sl = np.array([x0 - h * i for i in range(1, 7)])
    sr = np.array([x0 + h * i for i in range(1, 7)])
    pl = np.polyfit(sl - x0, [f(s) for s in sl], 4)
    pr = np.polyfit(sr - x0, [f(s) for s in sr], 4)
    d1l, d1r = pl[-2], pr[-2]
    d2l, d2r = 2 * pl[-3], 2 * pr[-3]
    d3l, d3r = 6 * pl[-4], 6 * pr[-4]
    assert abs(pl[-1] - pr[-1]) < 1e-12
    assert abs(d1l - d1r) < 1e-7
    assert abs(d2l - d2r) < 1e-3
    # the third derivative jumps by 8 pi^2 at 0 and by 4 pi^2 at +-1 (K1 is exactly C^2)
    jump = 8 * math.pi ** 2 if x0 == 0.0 else 4 * math.pi ** 2
    assert abs(abs(d3l - d3r) - jump) < 1e-2 * jump


def test_analytic_derivatives_match_fd(ora):
    for x in np.linspace(-0.99, 0.99, 199):
        if abs(x) < 1e-9:
            continue
        assert ora.dK1(x) == pytest.approx(_d(ora.K1, x, 1e-6, 1), abs=1e-8)
        assert ora.d2K1(x) == pytest.approx(_d(ora.K1, x, 1e-4, 2), abs=1e-5)


def _all_node_weights(ora, cfg, xp):
    nodes, w, d = ora.stencil(cfg, np.asarray(xp, float))
    out = {}
    for g in range(2):
        for o in range(8):
            out[(g,) + tuple(int(v) for v in nodes[g, o])] = w[g, o]
    return out


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("grid_face", [-1, 1])
def test_weights_c2_across_cell_faces(ora, axis, grid_face):
    """The 16 dual-grid weights, as functions of the particle position, stay C^2
    when the particle crosses a face of a G- or G+ cell (the stencil switches
    nodes there): values, first and second differences agree from both sides."""
    cfg = ora.config((8, 8, 8), 1.0)          # dx = 1: positions and derivatives in cell units
    rng = np.random.default_rng(11 + axis)
    for _ in range(5):
        base = 3.0 + rng.random(3)
        base[axis] = 4.0 + grid_face / 4.0   # X - k/4 integer: a face of grid k's cells
        e = np.zeros(3)
        e[axis] = 1.0
        h = 2e-4
        samples = {s: _all_node_weights(ora, cfg, base + s * h * e) for s in range(-6, 7)}
        keys = set().union(*[set(v) for v in samples.values()])
        for k in keys:
            f = np.array([samples[s].get(k, 0.0) for s in range(-6, 7)])
            t = np.arange(-6, 7) * h
            pl = np.polyfit(t[:6], f[:6], 3)
            pr = np.polyfit(t[7:], f[7:], 3)
            assert abs(np.polyval(pl, 0) - np.polyval(pr, 0)) < 1e-10
            assert abs(pl[-2] - pr[-2]) < 1e-6               # first derivative
            assert abs(2 * pl[-3] - 2 * pr[-3]) < 2e-3       # second derivative
