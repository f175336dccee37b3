"""GPU cell keys and sort against the CPU checker: bit-exact keys and permutation
(std::stable_sort on the same FP32 positions), including duplicates, positions
one ulp either side of cell faces, ragged sizes and the full 4.2M-particle
sand column."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_util import GpuRun, log

pytestmark = pytest.mark.gpu


def _gpu_sort(sc):
    import torch
    run = GpuRun(sc)
    n = sc.n
    keys = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    perm = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    s = run.ck.mpm_sort_keys(run.ctx.h, run.parts.c, keys.data_ptr(), perm.data_ptr(), run.stream)
    run.ck.check(s, "mpm_sort_keys")
    status = run.ck.mpm_sync(run.ctx.h, run.stream)
    k = keys.cpu().numpy().view(np.uint32)[:n].copy()
    p = perm.cpu().numpy().view(np.uint32)[:n].copy()
    run.close()
    return status, k, p


def _check(sc):
    status, k, p = _gpu_sort(sc)
    assert status == 0
    ok, bad = oracle.cell_keys(oracle.scene_config(sc), np.ascontiguousarray(sc.x.T))
    assert bad == 0
    assert np.array_equal(k, ok), "keys differ at %d positions" % int((k != ok).sum())
    op = oracle.stable_sort(ok)
    assert np.array_equal(p, op), "perm differs at %d positions" % int((p != op).sum())
    log("sort parity %s: n=%d exact" % (sc.name, sc.n))


def _faces_scene(seed, n_cells=(32, 32, 32)):
    sc = scenes.random_blob(seed, n_cells=n_cells, lo_cells=(3.0, 4.0, 5.0), ext_cells=(20, 17, 9))
    rng = np.random.default_rng(seed)
    x = sc.x.copy()
    n = x.shape[0]
    dx = sc.dx
    # duplicates: a quarter of the particles share a few positions
    dup = rng.choice(n, n // 4, replace=False)
    x[dup] = x[rng.choice(dup, 16)][rng.integers(0, 16, dup.size)]
    # one ulp either side of G- cell faces (X + 1/4 integer)
    face = rng.choice(n, n // 4, replace=False)
    axis = rng.integers(0, 3, face.size)
    Xf = np.floor(x[face, axis].astype(np.float64) / dx + 0.25) - 0.25
    xf = (Xf * dx).astype(np.float32)
    sgn = rng.integers(0, 2, face.size)
    x[face, axis] = np.where(sgn == 1, np.nextafter(xf, np.float32(1)), np.nextafter(xf, np.float32(-1)))
    sc.x = x
    return sc


@pytest.mark.parametrize("seed", [0, 1])
def test_sort_faces_and_duplicates(seed):
    _check(_faces_scene(seed))


def test_sort_exact_faces():
    sc = _faces_scene(5)
    dx = sc.dx
    # positions exactly on faces: floor puts them in the upper cell
    sc.x[:100, 0] = ((np.floor(sc.x[:100, 0] / dx + 0.25) - 0.25) * dx).astype(np.float32)
    _check(sc)


@pytest.mark.parametrize("builder", [scenes.cube_elastic, lambda: scenes.sand_column(scale=4)])
def test_sort_scenes(builder):
    _check(builder())


@pytest.mark.parametrize("n", [1, 2, 63, 65, 1000, 4097])
def test_sort_ragged_sizes(n):
    sc = scenes.random_blob(3, n_cells=(64, 64, 64), lo_cells=(4, 4, 4), ext_cells=(40, 40, 40))
    rng = np.random.default_rng(n)
    idx = rng.choice(sc.n, n, replace=False)
    for name in ("x", "v", "B", "F", "mat"):
        setattr(sc, name, getattr(sc, name)[idx])
    _check(sc)


def test_sort_shuffled_full_column():
    """The 4,194,304-particle sand column in a random order (worst case for the bucketing)."""
    sc = scenes.sand_column()
    rng = np.random.default_rng(7)
    order = rng.permutation(sc.n)
    for name in ("x", "v", "B", "F", "mat"):
        setattr(sc, name, getattr(sc, name)[order])
    _check(sc)
