"""The stress-scale workload on the GPU (~30.6M particles of sand stacks and an
elastic sphere on a 1024^3 virtual grid) checked on sampled outputs: one step of
the full scene, and the FP64 oracle run on the particles around a sample region
with a grid that covers only that region.  The state a step gives a particle
depends only on particles within two cells of it (the stencils of its nodes), so
for the particles of the region the oracle's result is exact once every particle
within three cells is included; the region lies away from the walls, so the small
grid needs none."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_util import TOL, GpuRun, log, nerr

pytestmark = pytest.mark.gpu


def _region_reference(sc, centre_cells, half=5, margin=4):
    X = sc.x.astype(np.float64) / sc.dx
    c = np.floor(np.asarray(centre_cells, np.float64)).astype(np.int64)
    lo, hi = c - half - margin, c + half + margin
    sel = np.all((X >= lo + 1) & (X < hi - 1), axis=1)
    idx = np.flatnonzero(sel)
    inner = np.all((X[idx] >= c - half) & (X[idx] < c + half), axis=1)
    cfg = oracle.config(tuple(int(v) for v in hi - lo), sc.dx, tuple(float(v) for v in lo * sc.dx), sc.gravity, 0)
    st = oracle.State(sc.x[idx], sc.v[idx], sc.B[idx], sc.F[idx], sc.mat[idx])
    status, _, _ = oracle.step(cfg, oracle.scene_materials(sc), st, sc.dt)
    assert status == 0
    return idx[inner], st, inner


def test_stress_scene_one_step_matches_oracle_on_sample_regions():
    sc = scenes.stress_scene()
    log("stress scene: %d particles (%d in the sphere)" % (sc.n, int((sc.mat == 1).sum())))
    run = GpuRun(sc)
    got = run.steps(sc.dt, 1)
    run.close()
    assert got["status"] == 0
    assert np.array_equal(np.sort(got["id"]), np.arange(sc.n))
    X = sc.x.astype(np.float64) / sc.dx
    sand = sc.mat == 0
    # sample regions: the sphere's centre, and inside the sand above the floor band
    ys = X[sand, 1]
    mid = sand & (X[:, 1] > 0.5 * ys.max()) & (X[:, 1] < 0.5 * ys.max() + 2)
    sand_centre = X[np.flatnonzero(mid)[len(np.flatnonzero(mid)) // 2]]
    sphere_centre = X[sc.mat == 1].mean(axis=0)
    for name, centre in (("sphere", sphere_centre), ("sand", sand_centre)):
        ids, st, inner = _region_reference(sc, centre)
        assert len(ids) > 500, name
        for k in ("x", "v", "F"):
            e = nerr(got[k][ids], getattr(st, k)[inner])
            log("stress scene, %s region (%d particles): %s %.2e" % (name, len(ids), k, e))
            assert e <= TOL, (name, k)
