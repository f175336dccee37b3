"""Particle storage order after a step, bit-exact: blocks in increasing virtual
block id, and inside a block the layered order of the P2G scatter (layer q holds
the q-th particle by index of every (half-cell octant, cell) bin, layers in
(octant, cell) order), or (octant, cell, index) order for a block whose largest
bin holds more than 16 particles.  G2P writes the new state at the positions P2G
assigned, so the ids of the stepped buffer, read in storage order, show the order
the transfer used.  The expected order is computed here from the input positions
with the same FP64 cell arithmetic (G- cell floor((x - origin)/dx + 1/4))."""
import numpy as np
import pytest

import scenes
from gpu_util import GpuRun, log

pytestmark = pytest.mark.gpu

LAYERS = 16


def expected_order(sc):
    x = sc.x.astype(np.float64)
    X = (x - np.asarray(sc.origin, np.float64)) * (1.0 / float(sc.dx))
    Xm = X + 0.25
    c = np.floor(Xm).astype(np.int64)
    up = (Xm - c) >= 0.5
    nb = [n // 4 + 1 for n in sc.n_cells]
    b = c >> 2
    vb = (b[:, 2] * nb[1] + b[:, 1]) * nb[0] + b[:, 0]
    cl = c & 3
    cell = cl[:, 2] * 16 + cl[:, 1] * 4 + cl[:, 0]
    octant = up[:, 0].astype(np.int64) | (up[:, 1].astype(np.int64) << 1) | (up[:, 2].astype(np.int64) << 2)
    binn = octant * 64 + cell
    idx = np.arange(len(x))
    out = []
    dense_blocks = 0
    for v in np.unique(vb):
        members = idx[vb == v]
        bins = binn[members]
        o = np.lexsort((members, bins))          # (bin, index)
        members, bins = members[o], bins[o]
        starts = np.r_[0, np.flatnonzero(np.diff(bins)) + 1]
        run = np.cumsum(np.r_[1, (np.diff(bins) != 0).astype(np.int64)]) - 1
        q = np.arange(len(members)) - starts[run]   # rank inside the bin
        if q.max() + 1 > LAYERS:
            dense_blocks += 1
            out.append(members)                      # (octant, cell, index)
        else:
            out.append(members[np.lexsort((bins, q))])   # (layer, octant, cell)
    return np.concatenate(out), dense_blocks


def _check(sc, want_dense):
    exp, dense = expected_order(sc)
    assert (dense > 0) == want_dense
    run = GpuRun(sc)
    got = run.steps(sc.dt, 1)
    assert got["status"] == 0
    ids = run.parts.read()["id"].astype(np.int64)
    run.close()
    log("%s: %d particles, %d dense blocks, order mismatches %d" % (sc.name, sc.n, dense, int((ids != exp).sum())))
    assert np.array_equal(ids, exp)


def test_layered_order_after_one_step():
    sc = scenes.random_blob(21, n_cells=(32, 32, 32), lo_cells=(7.3, 8.6, 9.1), ext_cells=(11, 9, 10), F_scale=0.02,
                            v_scale=0.1, dt=1e-4)
    _check(sc, want_dense=False)


def test_dense_block_keeps_octant_order():
    sc = scenes.random_blob(22, n_cells=(32, 32, 32), lo_cells=(7.3, 8.6, 9.1), ext_cells=(11, 9, 10), F_scale=0.02,
                            v_scale=0.1, dt=1e-4)
    # 24 particles inside one half-cell octant of one cell: that bin exceeds the
    # layer limit and its block falls back to the (octant, cell, index) order
    rng = np.random.default_rng(5)
    pick = rng.choice(sc.n, 24, replace=False)
    base = (np.array([12.0, 12.0, 12.0]) - 0.25 + 0.05) * sc.dx
    sc.x[pick] = (base + rng.random((24, 3)) * 0.4 * sc.dx).astype(np.float32)
    _check(sc, want_dense=True)


@pytest.mark.parametrize("dense", [False, True])
def test_kept_block_order_equals_order_from_scratch(dense):
    """A P2G whose input the context's own G2P wrote keeps the order of every block
    that G2P left unchanged (no particle entered, left or changed its (octant, cell)
    bin).  Particles moving about a cell per 100 steps leave some blocks unchanged
    each step and change others: the storage order after every step must be the one a
    run that orders every block from scratch (the state marked as changed on the
    host before each step) produces."""
    sc = scenes.random_blob(23, n_cells=(32, 32, 32), lo_cells=(7.3, 8.6, 9.1), ext_cells=(11, 9, 10), F_scale=0.02,
                            v_scale=0.3, dt=1e-3)
    if dense:
        rng = np.random.default_rng(6)
        pick = rng.choice(sc.n, 24, replace=False)
        base = (np.array([12.0, 12.0, 12.0]) - 0.25 + 0.05) * sc.dx
        sc.x[pick] = (base + rng.random((24, 3)) * 0.4 * sc.dx).astype(np.float32)
    kept = GpuRun(sc)
    fresh = GpuRun(sc)
    n_kept = n_changed = 0
    prev = None
    for k in range(12):
        a = kept.steps(sc.dt, 1)
        fresh.ck.check(fresh.ck.mpm_invalidate(fresh.ctx.h), "mpm_invalidate")
        b = fresh.steps(sc.dt, 1)
        assert a["status"] == 0 and b["status"] == 0
        ra = kept.parts.read()
        ia = ra["id"].astype(np.int64)
        ib = fresh.parts.read()["id"].astype(np.int64)
        assert np.array_equal(ia, ib), "step %d: %d positions differ" % (k + 1, int((ia != ib).sum()))
        # blocks the step left unchanged (the ones whose order a following P2G keeps)
        vb, binn = _block_bins(sc, ra["x"][np.argsort(ia)])
        if prev is not None:
            pvb, pbin = prev
            moved = (vb != pvb) | (binn != pbin)
            changed = set(np.unique(pvb[moved])) | set(np.unique(vb[moved]))
            blocks = set(np.unique(vb))
            n_changed += len(blocks & changed)
            n_kept += len(blocks - changed)
        prev = (vb, binn)
    log("kept block order%s: 11 steps, %d blocks left unchanged by their step, %d changed" % (
        " (dense block)" if dense else "", n_kept, n_changed))
    assert n_kept > 0 and n_changed > 0   # both the kept and the recomputed orders ran
    kept.close()
    fresh.close()


def _block_bins(sc, x):
    """Virtual block and (octant, cell) bin of each particle (FP64, as expected_order)."""
    X = (np.asarray(x, np.float64) - np.asarray(sc.origin, np.float64)) * (1.0 / float(sc.dx))
    Xm = X + 0.25
    c = np.floor(Xm).astype(np.int64)
    up = (Xm - c) >= 0.5
    nb = [n // 4 + 1 for n in sc.n_cells]
    b = c >> 2
    vb = (b[:, 2] * nb[1] + b[:, 1]) * nb[0] + b[:, 0]
    cl = c & 3
    octant = up[:, 0].astype(np.int64) | (up[:, 1].astype(np.int64) << 1) | (up[:, 2].astype(np.int64) << 2)
    return vb, octant * 64 + cl[:, 2] * 16 + cl[:, 1] * 4 + cl[:, 0]
