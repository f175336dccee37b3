"""The seeded scene generators: particle counts, determinism and domain."""
import numpy as np

import scenes


def test_cube_counts_and_determinism():
    a, b = scenes.cube_elastic(), scenes.cube_elastic()
    assert a.n == 32768 and np.array_equal(a.x, b.x)
    assert np.all(a.v[:, 1] == -1.0) and np.all(a.F == np.eye(3, dtype=np.float32))
    lo = a.x.min(axis=0)
    hi = a.x.max(axis=0)
    assert np.all(lo >= np.array([0.25, 0.35, 0.25]) - 1e-6) and np.all(hi <= np.array([0.75, 0.85, 0.75]) + 1e-6)


def test_sand_column_size_and_cells():
    sc = scenes.sand_column(scale=4)
    assert sc.n == 16 * 32 * 16 * 8
    X = sc.x.astype(np.float64) / sc.dx
    cells = np.floor(X).astype(np.int64)
    # stratified: exactly 8 particles in every dx-cell of the column
    _, counts = np.unique(cells[:, 0] + 1000 * cells[:, 1] + 1000000 * cells[:, 2], return_counts=True)
    assert np.all(counts == 8)
    assert X[:, 1].min() >= 2.0


def test_perturbed_and_floor_variants():
    a = scenes.cube_elastic_perturbed(1)
    b = scenes.cube_elastic_perturbed(1, floor_cells=2.5)
    assert np.allclose(np.std(a.F - np.eye(3), axis=0), 0.01, rtol=0.05)
    assert abs(b.x[:, 1].min() - 2.5 * b.dx) < 0.5 * b.dx
