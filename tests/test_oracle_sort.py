"""Pins of the oracle's cell keys and stable sort: keys recomputed here from the
definition with numpy, the permutation against numpy's stable argsort, and
positions placed one ulp either side of cell faces."""
import numpy as np
import pytest


def _numpy_keys(n_cells, dx, origin, x):
    X = (x.astype(np.float64) - np.asarray(origin)[:, None]) / dx
    c = np.floor(X + 0.25).astype(np.int64)
    NB = np.asarray(n_cells) // 4 + 1
    b = c >> 2
    vb = (b[2] * NB[1] + b[1]) * NB[0] + b[0]
    return ((vb << 6) | ((c[2] & 3) * 16 + (c[1] & 3) * 4 + (c[0] & 3))).astype(np.uint32)


@pytest.mark.parametrize("n_cells,dx,origin", [((32, 32, 32), 1 / 32, (0, 0, 0)),
                                                ((64, 16, 40), 1 / 64, (0.5, -0.25, 1.0)),
                                                ((256, 256, 256), 1 / 256, (0, 0, 0))])
def test_keys_and_stable_sort(ora, n_cells, dx, origin):
    rng = np.random.default_rng(0)
    n = 50000
    lo = np.asarray(origin)[:, None] + 0.25 * dx
    hi = np.asarray(origin)[:, None] + (np.asarray(n_cells)[:, None] - 0.25) * dx
    x = (lo + (hi - lo) * rng.random((3, n))).astype(np.float32)
    # many duplicates of a few cells so that stability matters, plus face +-1 ulp positions
    x[:, :2000] = x[:, :1][:, [0] * 2000]
    faces = (np.asarray(origin)[:, None] + (np.floor(x[:, 2000:6000].astype(np.float64) / dx) + 0.75) * dx)
    f32 = faces.astype(np.float32)
    x[:, 2000:4000] = np.nextafter(f32[:, :2000], np.float32(np.inf))
    x[:, 4000:6000] = np.nextafter(f32[:, 2000:], np.float32(-np.inf))
    x = np.clip(x, lo.astype(np.float32), np.nextafter(hi.astype(np.float32), np.float32(-np.inf)))
    cfg = ora.config(n_cells, dx, origin)
    keys, bad = ora.cell_keys(cfg, x)
    assert bad == 0
    assert np.array_equal(keys, _numpy_keys(n_cells, dx, origin, x))
    perm = ora.stable_sort(keys)
    assert np.array_equal(perm, np.argsort(keys, kind="stable").astype(np.uint32))


def test_out_of_domain_counted(ora):
    cfg = ora.config((16, 16, 16), 1 / 16)
    x = np.full((3, 5), 0.5, np.float32)
    x[0, 1] = 0.2 / 16           # below 1/4 cell
    x[1, 2] = 1.0 - 0.2 / 16     # above n - 1/4 cells
    x[2, 3] = np.nan
    keys, bad = ora.cell_keys(cfg, x)
    assert bad == 3
