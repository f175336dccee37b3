"""Job server on the GPU: every served job matches the FP64 checker's own
trajectory and is the same alone and in the mix, admission respects the memory
budget and submission order, and a job larger than the whole budget is refused."""
import functools
import time

import numpy as np
import pytest

import scenes
from gpu_util import TOL, log, nerr, oracle_state, oracle_step

pytestmark = pytest.mark.gpu


def _jobs():
    """Small jobs of both materials, sizes and grids (seeded)."""
    out = []
    for i, (seed, model, ext, n) in enumerate([(11, scenes.FIXED_COROTATED, (4, 4, 4), 16),
                                               (12, scenes.DRUCKER_PRAGER, (5, 3, 4), 16),
                                               (13, scenes.FIXED_COROTATED, (6, 6, 6), 32),
                                               (14, scenes.DRUCKER_PRAGER, (8, 4, 8), 32),
                                               (15, scenes.FIXED_COROTATED, (3, 7, 5), 16)]):
        sc = scenes.random_blob(seed, n_cells=(n, n, n), lo_cells=(5.0, 5.0, 5.0), ext_cells=ext, model=model,
                                v_scale=0.3, B_scale=1.0, F_scale=0.01, gravity=(0.0, -9.8, 0.0), bc_band=2,
                                dt=1e-4)
        out.append(sc)
    for spec in (scenes.serving_workload(seed=4, n_jobs=8)[k] for k in (1, 7)):
        spec.nsteps = 12
        out.append(scenes.serving_job(spec))
    return out


def _alone(sc, nsteps):
    import torch
    from paper_2412_10399_amd import ckmpm
    ctx = ckmpm.Context(ckmpm.job_config(sc), ckmpm.scene_materials(sc))
    parts = ckmpm.particles_from_scene(sc, "cuda:0")
    s = torch.cuda.current_stream()
    ckmpm.check(ckmpm.mpm_step(ctx.h, parts.c, sc.dt, nsteps, s))
    ckmpm.check(ckmpm.mpm_sync(ctx.h, s))
    out = parts.read_by_id()
    ctx.close()
    return out


@functools.lru_cache(maxsize=None)
def _oracle_final(k, nsteps):
    """The checker's FP64 state of job k of _jobs() after nsteps steps."""
    sc = _jobs()[k]
    st = oracle_state(dict(x=sc.x, v=sc.v, B=sc.B, F=sc.F))
    for _ in range(nsteps):
        oracle_step(sc, st, sc.dt, grids=False)
    return st


def _check_oracle(tag, got, st):
    """x, v, F of a served job (read back in particle-id order) against the checker."""
    assert np.array_equal(got["id"], np.arange(st.n))
    errs = {name: nerr(got[name], getattr(st, name)) for name in ("x", "v", "F")}
    log("%s vs checker: %s" % (tag, " ".join("%s=%.2e" % kv for kv in errs.items())))
    for name, e in errs.items():
        assert e <= TOL, "%s: %s error %.3e" % (tag, name, e)


def _collect(srv, jids, timeout=120.0):
    """Client loop: poll, read and release finished jobs until all are collected."""
    from paper_2412_10399_amd import ckmpm
    got, infos = {}, {}
    t0 = time.time()
    while len(got) < len(jids):
        srv.poll()
        for j in jids:
            if j in got:
                continue
            info = srv.info(j)
            if info.state in (ckmpm.MPM_JOB_DONE, ckmpm.MPM_JOB_FAILED):
                infos[j] = (info.state, info.status, info.t_submit, info.t_admit, info.t_done, info.steps_done)
                got[j] = srv.read(j)
                srv.release(j)
        assert time.time() - t0 < timeout, "jobs did not finish"
        time.sleep(0.0005)
    return got, infos


def _compare(a, b):
    for name in ("x", "v", "F"):
        assert nerr(a[name], b[name]) < TOL, name
    assert np.array_equal(a["id"], b["id"])


@pytest.mark.parametrize("grouped", [False, True])
@pytest.mark.parametrize("spl", [2, 4])
def test_jobs_alone_equal_jobs_in_the_mix(spl, grouped):
    """Per-job launches on several streams, or (grouped) one launch per phase for all
    active jobs."""
    from paper_2412_10399_amd import ckmpm
    jobs = _jobs()
    nsteps = 12
    ref = [_alone(sc, nsteps) for sc in jobs]
    srv = ckmpm.Server(memory_budget=1 << 30, max_jobs=8, n_streams=3, steps_per_launch=spl, grouped=grouped)
    jids = [srv.submit_scene(sc, nsteps) for sc in jobs]
    got, infos = _collect(srv, jids)
    for k, j in enumerate(jids):
        state, status, *_ , steps = infos[j]
        assert state == ckmpm.MPM_JOB_DONE and status == 0 and steps == nsteps
        _check_oracle("job %d (%d particles, %s, %d steps/launch)" % (k, jobs[k].n, "grouped" if grouped else
                                                                      "per-job", spl), got[j], _oracle_final(k, nsteps))
        _compare(got[j], ref[k])
    lat = srv.step_latencies()
    assert len(lat) == nsteps * len(jobs) and min(lat) > 0.0
    log("served %d jobs, step latency p50 %.1f us" % (len(jobs), 1e6 * float(np.median(lat))))
    srv.close()


@pytest.mark.parametrize("grouped", [False, True])
def test_low_memory_budget_admits_one_job_at_a_time(grouped):
    from paper_2412_10399_amd import ckmpm
    jobs = _jobs()[:4]
    nsteps = 6
    fps = [ckmpm.mpm_footprint(ckmpm.job_config(sc), sc.n) for sc in jobs]
    budget = max(fps) + min(fps) // 2          # never two of these jobs at once
    ref = [_alone(sc, nsteps) for sc in jobs]
    srv = ckmpm.Server(memory_budget=budget, max_jobs=8, n_streams=2, steps_per_launch=2, grouped=grouped)
    jids = [srv.submit_scene(sc, nsteps) for sc in jobs]
    got, infos = _collect(srv, jids)
    admits = [infos[j][3] for j in jids]
    dones = [infos[j][4] for j in jids]
    assert admits == sorted(admits)                     # submission order
    for k in range(1, len(jids)):
        assert admits[k] >= dones[k - 1]               # one resident job at a time
    for k, j in enumerate(jids):
        assert infos[j][0] == ckmpm.MPM_JOB_DONE
        _compare(got[j], ref[k])
    srv.close()


def test_job_larger_than_budget_is_refused_and_empty_job_finishes():
    import torch
    from paper_2412_10399_amd import ckmpm
    sc = _jobs()[0]
    fp = ckmpm.mpm_footprint(ckmpm.job_config(sc), sc.n)
    srv = ckmpm.Server(memory_budget=fp // 2, max_jobs=2, n_streams=1, steps_per_launch=2)
    state = torch.from_numpy(ckmpm.state_planes(sc.x, sc.v, sc.B, sc.F)).cuda()
    with pytest.raises(ckmpm.CkMpmError) as e:
        srv.submit(ckmpm.job_config(sc), ckmpm.scene_materials(sc), state, 4, sc.dt)
    assert e.value.status == ckmpm.MPM_E_CAPACITY
    srv.close()
    srv = ckmpm.Server(memory_budget=2 * fp, max_jobs=2, n_streams=1, steps_per_launch=2)
    j = srv.submit(ckmpm.job_config(sc), ckmpm.scene_materials(sc), state, 0, sc.dt)
    srv.drain()
    info = srv.info(j)
    assert info.state == ckmpm.MPM_JOB_DONE and info.steps_done == 0
    out = srv.read(j)
    assert np.array_equal(out["x"], sc.x) and np.array_equal(out["v"], sc.v)
    srv.release(j)
    srv.close()


def test_grouped_server_uneven_steps_and_refusals():
    """Grouped rounds with jobs of different step counts (each round runs a job only
    for the steps it has left), a zero-step job, and refusal of a job the grouped
    launches cannot run (the quadratic comparison kernel)."""
    import torch
    from paper_2412_10399_amd import ckmpm
    jobs = _jobs()[:3]
    steps = [6, 10, 0]
    ref = [_alone(sc, k) if k else None for sc, k in zip(jobs, steps)]
    srv = ckmpm.Server(memory_budget=1 << 30, max_jobs=8, n_streams=1, steps_per_launch=4, grouped=True)
    jids = [srv.submit_scene(sc, k) for sc, k in zip(jobs, steps)]
    got, infos = _collect(srv, jids)
    for k, j in enumerate(jids):
        assert infos[j][0] == ckmpm.MPM_JOB_DONE and infos[j][5] == steps[k]
        if steps[k]:
            _compare(got[j], ref[k])
        else:
            assert np.array_equal(got[j]["x"], jobs[k].x)
    sc = jobs[0]
    cfg = ckmpm.job_config(sc)
    cfg.flags = ckmpm.MPM_FLAG_QUADRATIC
    state = torch.from_numpy(ckmpm.state_planes(sc.x, sc.v, sc.B, sc.F)).cuda()
    with pytest.raises(ckmpm.CkMpmError) as e:
        srv.submit(cfg, ckmpm.scene_materials(sc), state, 4, sc.dt)
    assert e.value.status == ckmpm.MPM_E_INVALID
    srv.close()
