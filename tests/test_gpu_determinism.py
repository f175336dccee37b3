"""Deterministic mode (mpm_config.deterministic = 1) on the GPU: bitwise equal runs,
bitwise resume from a copy of the particle state, bitwise equal phase calls and
mpm_step, the same FP64-checker parity as the default mode, and served jobs bitwise
equal alone and in the mix (per-job and grouped servers)."""
import numpy as np
import pytest

import scenes
from gpu_util import TOL, GpuRun, log, nerr, oracle_state, oracle_step

pytestmark = pytest.mark.gpu


def _raw(run):
    """Current buffer (all state planes) and ids in storage order, as host arrays."""
    p = run.parts
    cur = p.current
    return p.state[cur, :, :p.n].cpu().numpy().copy(), p.ids[cur, :p.n].cpu().numpy().copy()


def _bitwise(a, b):
    return np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("name", ["sand_column_quarter", "cube_elastic_floor"])
def test_two_runs_bitwise_equal(name):
    sc = scenes.sand_column(scale=4) if name == "sand_column_quarter" else scenes.cube_elastic_perturbed(
        1, floor_cells=2.5)
    a = GpuRun(sc, deterministic=True)
    b = GpuRun(sc, deterministic=True)
    for k in range(6):
        ga = a.phase_step(sc.dt)
        gb = b.phase_step(sc.dt)
        assert ga["status"] == 0 and gb["status"] == 0
        for key in ("m", "p", "vt"):
            assert _bitwise(ga[key], gb[key]), "step %d grid %s differs" % (k + 1, key)
    ga = a.steps(sc.dt, 8)
    gb = b.steps(sc.dt, 8)
    assert ga["status"] == 0 and gb["status"] == 0
    sa, ia = _raw(a)
    sb, ib = _raw(b)
    assert np.array_equal(ia, ib)
    assert _bitwise(sa, sb)
    log("%s: two deterministic runs of 14 steps bitwise equal" % name)
    a.close()
    b.close()


def test_phase_calls_and_mpm_step_bitwise_equal():
    sc = scenes.cube_elastic_perturbed(1)
    a = GpuRun(sc, deterministic=True)
    b = GpuRun(sc, deterministic=True)
    for _ in range(4):
        a.phase_step(sc.dt, want_grids=False)
    b.steps(sc.dt, 4)
    sa, ia = _raw(a)
    sb, ib = _raw(b)
    assert np.array_equal(ia, ib) and _bitwise(sa, sb)
    assert a.ck.mpm_current_buffer(a.ctx.h) == a.parts.current
    assert b.ck.mpm_current_buffer(b.ctx.h) == b.parts.current == 0   # four flips
    a.close()
    b.close()


def test_resume_from_particle_state_is_bitwise():
    """Checkpoint the particle SoA (all state planes and ids, as stored) after 5 steps, resume
    it in a fresh context and compare 7 further steps with the uninterrupted run."""
    import torch
    sc = scenes.sand_column(scale=4)
    a = GpuRun(sc, deterministic=True)
    assert a.ck.mpm_current_buffer(a.ctx.h) == -1
    assert a.steps(sc.dt, 5)["status"] == 0
    assert a.ck.mpm_current_buffer(a.ctx.h) == a.parts.current == 1
    ck_state, ck_ids = _raw(a)
    assert a.steps(sc.dt, 7)["status"] == 0
    b = GpuRun(sc, deterministic=True)
    cur = b.parts.current
    b.parts.state[cur, :, :sc.n].copy_(torch.from_numpy(ck_state))
    b.parts.ids[cur, :sc.n].copy_(torch.from_numpy(ck_ids))
    torch.cuda.synchronize()
    assert b.ck.mpm_invalidate(b.ctx.h) == 0
    assert b.steps(sc.dt, 7)["status"] == 0
    sa, ia = _raw(a)
    sb, ib = _raw(b)
    assert np.array_equal(ia, ib)
    assert _bitwise(sa, sb)
    log("resume after 5 steps: 7 further steps bitwise equal to the uninterrupted run")
    a.close()
    b.close()


def test_deterministic_mode_parity_with_the_checker():
    """Ten steps of the reduced sand column against the FP64 checker's trajectory, and
    against the default mode (float-atomic cross-block sums) to rounding."""
    sc = scenes.sand_column(scale=4)
    run = GpuRun(sc, deterministic=True)
    ref = GpuRun(sc)
    st = oracle_state(dict(x=sc.x, v=sc.v, B=sc.B, F=sc.F))
    for k in range(10):
        got = run.phase_step(sc.dt)
        dflt = ref.phase_step(sc.dt, want_grids=False)
        assert got["status"] == 0
        _, g = oracle_step(sc, st, sc.dt)
        em, ep = nerr(got["m"], g["m"]), nerr(got["p"], g["p"])
        emv = nerr(got["m"][..., None].astype(np.float64) * got["vt"], g["m"][..., None] * g["v"])
        errs = {name: nerr(got[name], getattr(st, name)) for name in ("x", "v", "F")}
        log("deterministic step %d: grid m=%.2e p=%.2e m*v~=%.2e particles %s" % (
            k + 1, em, ep, emv, " ".join("%s=%.2e" % kv for kv in errs.items())))
        assert em <= TOL and ep <= TOL and emv <= TOL
        for name, e in errs.items():
            assert e <= TOL, name
        for name in ("x", "v", "F"):
            assert nerr(got[name], dflt[name]) < 1e-6
    run.close()
    ref.close()


def _served(jobs, nsteps, grouped, max_jobs, deterministic=True):
    import time

    from paper_2412_10399_amd import ckmpm
    import torch
    srv = ckmpm.Server(memory_budget=1 << 30, max_jobs=max_jobs, n_streams=3, steps_per_launch=4, grouped=grouped)
    jids = []
    for sc in jobs:
        state = torch.from_numpy(ckmpm.state_planes(sc.x, sc.v, sc.B, sc.F)).cuda()
        cfg = ckmpm.job_config(sc, deterministic=deterministic)
        jids.append(srv.submit(cfg, ckmpm.scene_materials(sc), state, nsteps, sc.dt))
    t0 = time.time()
    out = {}
    while len(out) < len(jids):
        srv.poll()
        for k, j in enumerate(jids):
            if k in out:
                continue
            info = srv.info(j)
            if info.state in (ckmpm.MPM_JOB_DONE, ckmpm.MPM_JOB_FAILED):
                assert info.state == ckmpm.MPM_JOB_DONE and info.status == 0
                n = int(info.n)
                st = torch.empty((ckmpm.MPM_STATE_PLANES, n), dtype=torch.float32, device="cuda")
                ids = torch.empty(n, dtype=torch.int32, device="cuda")
                ckmpm.check(ckmpm.mpm_server_job_read(srv.h, j, st.data_ptr(), ids.data_ptr()))
                out[k] = (st.cpu().numpy(), ids.cpu().numpy())
                srv.release(j)
        assert time.time() - t0 < 120, "jobs did not finish"
        time.sleep(0.0005)
    srv.close()
    return [out[k] for k in range(len(jobs))]


@pytest.mark.parametrize("grouped", [False, True])
def test_served_jobs_bitwise_alone_and_in_the_mix(grouped):
    jobs = []
    for seed, model, ext in [(21, scenes.FIXED_COROTATED, (5, 4, 6)), (22, scenes.DRUCKER_PRAGER, (6, 3, 5)),
                             (23, scenes.FIXED_COROTATED, (8, 6, 7)), (24, scenes.DRUCKER_PRAGER, (4, 7, 4))]:
        jobs.append(scenes.random_blob(seed, n_cells=(32, 32, 32), lo_cells=(6.0, 5.0, 7.0), ext_cells=ext, model=model,
                                       v_scale=0.3, B_scale=1.0, F_scale=0.01, gravity=(0.0, -9.8, 0.0), bc_band=2,
                                       dt=1e-4))
    nsteps = 8
    mix = _served(jobs, nsteps, grouped, max_jobs=8)
    for k, sc in enumerate(jobs):
        alone = _served([sc], nsteps, grouped, max_jobs=1)[0]
        assert np.array_equal(mix[k][1], alone[1]), "job %d order" % k
        assert _bitwise(mix[k][0], alone[0]), "job %d state" % k
    log("%s server: %d deterministic jobs bitwise equal alone and in the mix" % (
        "grouped" if grouped else "per-job", len(jobs)))
