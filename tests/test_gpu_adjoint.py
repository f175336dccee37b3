"""The differentiable step on the GPU (include/ckmpm_adjoint.h) against the FP64
oracle: one forward step, one reverse-mode step with random cotangents (also with
the particles shuffled, which takes the scatters' direct path), rollout
gradients of the differentiation workload (65,536 particles, 64 steps, checkpoints
every 8 steps) against the oracle's adjoint, 32 random directional derivatives
against central differences of the oracle's forward rollout, and the block-sparse
grid pool (a 256^3 grid holding only the touched blocks, pool overflow)."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_util import TOL, log, nerr

pytestmark = pytest.mark.gpu


def _ctx(sc, mode=None):
    """Context for scene sc: the pool of ckmpm.scene_config (mode None), a slot for
    every block of the lattice ("direct") or one block fewer, which makes every call
    mark its blocks and take slots ("sparse")."""
    from paper_2412_10399_amd import ckmpm, diff
    nb = int(np.prod([c // 4 + 1 for c in sc.n_cells]))
    mb = {None: None, "direct": nb, "sparse": nb - 1}[mode]
    return diff.AdContext(ckmpm.scene_config(sc, max_blocks=mb), ckmpm.scene_materials(sc)[0])


def _state(sc, x=None, v=None, B=None, F=None):
    import torch
    from paper_2412_10399_amd import ckmpm
    p = ckmpm.state_planes(sc.x if x is None else x, sc.v if v is None else v, sc.B if B is None else B,
                           sc.F if F is None else F)
    return torch.from_numpy(p).cuda()


def _unpack(planes):
    from paper_2412_10399_amd import ckmpm
    return ckmpm.unpack_state(planes.cpu().numpy())


def _fc_scene(seed, near_wall=False):
    sc = scenes.random_blob(seed, n_cells=(16, 16, 16), lo_cells=(2.2, 2.4, 5.1) if near_wall else (5.3, 5.6, 4.2),
                            ext_cells=(6, 4, 5), model=scenes.FIXED_COROTATED, v_scale=0.5, B_scale=2.0,
                            F_scale=0.05, gravity=(0.3, -9.8, 0.1), bc_band=2, dt=1e-4, E=5e4)
    rng = np.random.default_rng(seed + 7)
    sc.logE = (np.log(5e4) + 0.2 * rng.standard_normal(sc.n)).astype(np.float32)
    return sc


@pytest.mark.parametrize("mode", ["direct", "sparse"])
@pytest.mark.parametrize("near_wall", [False, True])
def test_forward_step_matches_oracle(near_wall, mode):
    import torch
    from paper_2412_10399_amd import ckmpm
    sc = _fc_scene(31, near_wall)
    ad = _ctx(sc, mode)
    s0 = _state(sc)
    logE = torch.from_numpy(sc.logE).cuda()
    out = torch.empty_like(s0)
    stream = torch.cuda.current_stream()
    ckmpm.check(ckmpm.mpm_ad_forward(ad.h, sc.n, sc.n, s0.data_ptr(), logE.data_ptr(), out.data_ptr(), sc.dt, stream))
    ckmpm.check(ckmpm.mpm_ad_sync(ad.h, stream))
    got = _unpack(out)
    st = oracle.State(sc.x, sc.v, sc.B, sc.F, sc.mat, sc.logE)
    status, _, _ = oracle.step(oracle.scene_config(sc), oracle.scene_materials(sc), st, sc.dt)
    assert status == 0
    for k in ("x", "v", "F"):
        e = nerr(got[k], getattr(st, k))
        log("differentiable forward step (near wall %s, %s pool): %s %.2e" % (near_wall, mode, k, e))
        assert e <= TOL, k
    assert nerr(got["B"], st.B) <= 10 * TOL
    ad.close()


@pytest.mark.parametrize("mode", ["direct", "sparse"])
@pytest.mark.parametrize("near_wall", [False, True])
def test_backward_step_matches_oracle_adjoint(near_wall, mode):
    import torch
    from paper_2412_10399_amd import ckmpm
    sc = _fc_scene(32, near_wall)
    ad = _ctx(sc, mode)
    n = sc.n
    rng = np.random.default_rng(3)
    cot = [rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), 64 * rng.standard_normal((n, 3, 3)),
           rng.standard_normal((n, 3, 3))]
    st = oracle.State(sc.x, sc.v, sc.B, sc.F, sc.mat, sc.logE)
    status, ref = oracle.step_vjp(oracle.scene_config(sc), oracle.scene_materials(sc), st, sc.dt, *cot)
    assert status == 0
    s0 = _state(sc)
    logE = torch.from_numpy(sc.logE).cuda()
    cot_out = torch.from_numpy(np.concatenate([cot[0].T, cot[1].T, cot[2].reshape(n, 9).T, cot[3].reshape(n, 9).T,
                                               np.zeros((3, n))])
                               .astype(np.float32)).cuda().contiguous()
    cot_in = torch.empty_like(cot_out)
    lcot = torch.zeros(n, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    ckmpm.check(ckmpm.mpm_ad_backward(ad.h, n, n, s0.data_ptr(), logE.data_ptr(), cot_out.data_ptr(),
                                      cot_in.data_ptr(), lcot.data_ptr(), sc.dt, stream))
    ckmpm.check(ckmpm.mpm_ad_sync(ad.h, stream))
    g = cot_in.cpu().numpy().astype(np.float64)
    assert np.array_equal(g[24:27], g[0:3])   # the position x + r: one cotangent for both
    got = dict(x=g[0:3].T, v=g[3:6].T, B=g[6:15].T.reshape(n, 3, 3), F=g[15:24].T.reshape(n, 3, 3),
               logE=lcot.cpu().numpy())
    for k in ("x", "v", "B", "F", "logE"):
        e = nerr(got[k], ref[k])
        log("reverse step (near wall %s, %s pool): d/d%s %.2e" % (near_wall, mode, k, e))
        assert e <= 1e-4, k
    ad.close()


def test_shuffled_particles_take_the_direct_scatter():
    """Particles in random order: every workgroup's node box spans the body and
    exceeds the scatter tile, so both scatters add straight into the grid; forward
    and reverse step still match the oracle."""
    import torch
    from paper_2412_10399_amd import ckmpm
    sc = scenes.random_blob(35, n_cells=(16, 16, 16), lo_cells=(3.2, 3.4, 3.1), ext_cells=(10, 8, 9),
                            model=scenes.FIXED_COROTATED, v_scale=0.5, B_scale=2.0, F_scale=0.05,
                            gravity=(0.3, -9.8, 0.1), bc_band=2, dt=1e-4, E=5e4)
    rng = np.random.default_rng(36)
    perm = rng.permutation(sc.n)
    sc.x, sc.v, sc.B, sc.F, sc.mat = sc.x[perm], sc.v[perm], sc.B[perm], sc.F[perm], sc.mat[perm]
    sc.logE = (np.log(5e4) + 0.2 * rng.standard_normal(sc.n)).astype(np.float32)
    # a 256-particle workgroup's box needs more than the 5120-word tile
    X = sc.x[:256].astype(np.float64) / sc.dx
    span = np.floor(X.max(0) + 0.25) - np.floor(X.min(0) - 0.25) + 2
    assert 2 * np.prod(span) * 3 > 5120
    ad = _ctx(sc)
    n = sc.n
    s0 = _state(sc)
    logE = torch.from_numpy(sc.logE).cuda()
    stream = torch.cuda.current_stream()
    out = torch.empty_like(s0)
    ckmpm.check(ckmpm.mpm_ad_forward(ad.h, n, n, s0.data_ptr(), logE.data_ptr(), out.data_ptr(), sc.dt, stream))
    ckmpm.check(ckmpm.mpm_ad_sync(ad.h, stream))
    got = _unpack(out)
    st = oracle.State(sc.x, sc.v, sc.B, sc.F, sc.mat, sc.logE)
    status, _, _ = oracle.step(oracle.scene_config(sc), oracle.scene_materials(sc), st, sc.dt)
    assert status == 0
    for k in ("x", "v", "F"):
        e = nerr(got[k], getattr(st, k))
        log("shuffled forward step: %s %.2e" % (k, e))
        assert e <= TOL, k
    cot = [rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), 64 * rng.standard_normal((n, 3, 3)),
           rng.standard_normal((n, 3, 3))]
    st = oracle.State(sc.x, sc.v, sc.B, sc.F, sc.mat, sc.logE)
    status, ref = oracle.step_vjp(oracle.scene_config(sc), oracle.scene_materials(sc), st, sc.dt, *cot)
    assert status == 0
    cot_out = torch.from_numpy(np.concatenate([cot[0].T, cot[1].T, cot[2].reshape(n, 9).T, cot[3].reshape(n, 9).T,
                                               np.zeros((3, n))])
                               .astype(np.float32)).cuda().contiguous()
    cot_in = torch.empty_like(cot_out)
    lcot = torch.zeros(n, dtype=torch.float32, device="cuda")
    ckmpm.check(ckmpm.mpm_ad_backward(ad.h, n, n, s0.data_ptr(), logE.data_ptr(), cot_out.data_ptr(),
                                      cot_in.data_ptr(), lcot.data_ptr(), sc.dt, stream))
    ckmpm.check(ckmpm.mpm_ad_sync(ad.h, stream))
    g = cot_in.cpu().numpy().astype(np.float64)
    assert np.array_equal(g[24:27], g[0:3])   # the position x + r: one cotangent for both
    got = dict(x=g[0:3].T, v=g[3:6].T, B=g[6:15].T.reshape(n, 3, 3), F=g[15:24].T.reshape(n, 3, 3),
               logE=lcot.cpu().numpy())
    for k in ("x", "v", "B", "F", "logE"):
        e = nerr(got[k], ref[k])
        log("shuffled reverse step: d/d%s %.2e" % (k, e))
        assert e <= 1e-4, k
    ad.close()


def _one_step_both_ways(sc, ad, cot):
    """Forward and reverse step of scene sc on context ad: (state after, cotangents)."""
    import torch
    from paper_2412_10399_amd import ckmpm
    n = sc.n
    s0 = _state(sc)
    logE = torch.from_numpy(sc.logE).cuda()
    stream = torch.cuda.current_stream()
    out = torch.empty_like(s0)
    ckmpm.check(ckmpm.mpm_ad_forward(ad.h, n, n, s0.data_ptr(), logE.data_ptr(), out.data_ptr(), sc.dt, stream))
    ckmpm.check(ckmpm.mpm_ad_sync(ad.h, stream))
    cot_out = torch.from_numpy(np.concatenate([cot[0].T, cot[1].T, cot[2].reshape(n, 9).T, cot[3].reshape(n, 9).T,
                                               np.zeros((3, n))])
                               .astype(np.float32)).cuda().contiguous()
    cot_in = torch.empty_like(cot_out)
    lcot = torch.zeros(n, dtype=torch.float32, device="cuda")
    ckmpm.check(ckmpm.mpm_ad_backward(ad.h, n, n, s0.data_ptr(), logE.data_ptr(), cot_out.data_ptr(),
                                      cot_in.data_ptr(), lcot.data_ptr(), sc.dt, stream))
    ckmpm.check(ckmpm.mpm_ad_sync(ad.h, stream))
    g = cot_in.cpu().numpy().astype(np.float64)
    grads = dict(x=g[0:3].T, v=g[3:6].T, B=g[6:15].T.reshape(n, 3, 3), F=g[15:24].T.reshape(n, 3, 3),
                 logE=lcot.cpu().numpy())
    return _unpack(out), grads


def test_large_grid_holds_only_the_touched_blocks():
    """The same body on a 16^3 grid and, moved 120 cells in, on a 256^3 grid whose
    dense grids would take about 1.9 GB: the context takes tens of MB, and forward
    and reverse step agree with the small grid's (positions quantised to 2^-16
    cells, so that both grids see the same cell coordinates exactly) and with the
    oracle."""
    import dataclasses
    import torch
    from paper_2412_10399_amd import ckmpm, diff
    sc = _fc_scene(37)
    q = 2.0 ** 16 / sc.dx
    sc.x = (np.round(sc.x.astype(np.float64) * q) / q).astype(np.float32)
    shift = 120 * sc.dx
    big = dataclasses.replace(sc, n_cells=(256, 256, 256), origin=(-shift, -shift, -shift))
    n = sc.n
    rng = np.random.default_rng(38)
    cot = [rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), 64 * rng.standard_normal((n, 3, 3)),
           rng.standard_normal((n, 3, 3))]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ad_big = diff.AdContext(ckmpm.scene_config(big), ckmpm.scene_materials(big)[0])
    taken = free0 - torch.cuda.mem_get_info()[0]
    log("256^3 differentiable context: %.1f MB of device memory (dense grids: %.0f MB)"
        % (taken / 1e6, 14 * 2 * 257 ** 3 * 4 / 1e6))
    assert taken < 64 * 2 ** 20
    got_big, grad_big = _one_step_both_ways(big, ad_big, cot)
    ad_big.close()
    ad = _ctx(sc)
    got, grad = _one_step_both_ways(sc, ad, cot)
    ad.close()
    for k in ("x", "v", "B", "F"):
        e = nerr(got_big[k], got[k])
        log("256^3 vs 16^3 forward step: %s %.2e" % (k, e))
        assert e <= 1e-6, k
    for k in ("x", "v", "B", "F", "logE"):
        e = nerr(grad_big[k], grad[k])
        log("256^3 vs 16^3 reverse step: d/d%s %.2e" % (k, e))
        assert e <= 1e-6, k
    st = oracle.State(sc.x, sc.v, sc.B, sc.F, sc.mat, sc.logE)
    status, _, _ = oracle.step(oracle.scene_config(sc), oracle.scene_materials(sc), st, sc.dt)
    assert status == 0
    for k in ("x", "v", "F"):
        assert nerr(got_big[k], getattr(st, k)) <= TOL, k
    st = oracle.State(sc.x, sc.v, sc.B, sc.F, sc.mat, sc.logE)
    status, ref = oracle.step_vjp(oracle.scene_config(sc), oracle.scene_materials(sc), st, sc.dt, *cot)
    assert status == 0
    for k in ("x", "v", "B", "F", "logE"):
        assert nerr(grad_big[k], ref[k]) <= 1e-4, k


def test_pool_overflow_is_reported_and_the_next_call_recovers():
    """A one-block pool per grid: a body that needs more blocks makes the call
    report MPM_E_CAPACITY; a single particle at a block's centre (one block on each
    grid) then steps on the same context as on one with room to spare."""
    import torch
    from paper_2412_10399_amd import ckmpm, diff
    sc = _fc_scene(39)
    ad = diff.AdContext(ckmpm.scene_config(sc, max_blocks=1), ckmpm.scene_materials(sc)[0])
    s0 = _state(sc)
    logE = torch.from_numpy(sc.logE).cuda()
    out = torch.empty_like(s0)
    stream = torch.cuda.current_stream()
    ckmpm.check(ckmpm.mpm_ad_forward(ad.h, sc.n, sc.n, s0.data_ptr(), logE.data_ptr(), out.data_ptr(), sc.dt,
                                     stream))
    assert ckmpm.mpm_ad_sync(ad.h, stream) == ckmpm.MPM_E_CAPACITY
    one = _single_particle(sc, (4 * 2 + 2.0) * sc.dx)
    rng = np.random.default_rng(40)
    cot = [rng.standard_normal((1, 3)), rng.standard_normal((1, 3)), 64 * rng.standard_normal((1, 3, 3)),
           rng.standard_normal((1, 3, 3))]
    got, grad = _one_step_both_ways(one, ad, cot)
    ad.close()
    roomy = _ctx(one)
    want, want_grad = _one_step_both_ways(one, roomy, cot)
    roomy.close()
    for k in ("x", "v", "B", "F"):
        assert nerr(got[k], want[k]) <= 1e-6, k
    for k in ("x", "v", "B", "F", "logE"):
        assert nerr(grad[k], want_grad[k]) <= 1e-6, k
    log("one-block pool: overflow reported, single-particle step after it matches")


def test_particle_outside_the_domain_is_reported():
    """A particle closer than a quarter cell to the lattice's low face: forward and
    reverse call report MPM_E_DOMAIN, the forward call passes it through unchanged
    and the other particles match a run without it."""
    import dataclasses
    import torch
    from paper_2412_10399_amd import ckmpm
    sc = _fc_scene(41)
    sc.x[0] = np.float32(0.1 * sc.dx)
    ad = _ctx(sc)
    n = sc.n
    s0 = _state(sc)
    logE = torch.from_numpy(sc.logE).cuda()
    out = torch.empty_like(s0)
    stream = torch.cuda.current_stream()
    ckmpm.check(ckmpm.mpm_ad_forward(ad.h, n, n, s0.data_ptr(), logE.data_ptr(), out.data_ptr(), sc.dt, stream))
    assert ckmpm.mpm_ad_sync(ad.h, stream) == ckmpm.MPM_E_DOMAIN
    assert torch.equal(out[:, 0], s0[:, 0])
    cot_out = torch.ones_like(s0)
    cot_in = torch.empty_like(s0)
    lcot = torch.zeros(n, dtype=torch.float32, device="cuda")
    ckmpm.check(ckmpm.mpm_ad_backward(ad.h, n, n, s0.data_ptr(), logE.data_ptr(), cot_out.data_ptr(),
                                      cot_in.data_ptr(), lcot.data_ptr(), sc.dt, stream))
    assert ckmpm.mpm_ad_sync(ad.h, stream) == ckmpm.MPM_E_DOMAIN
    ckmpm.check(ckmpm.mpm_ad_sync(ad.h, stream))   # the status word was cleared
    rest = dataclasses.replace(sc, x=sc.x[1:], v=sc.v[1:], B=sc.B[1:], F=sc.F[1:], mat=sc.mat[1:], logE=sc.logE[1:])
    s1 = _state(rest)
    out1 = torch.empty_like(s1)
    ckmpm.check(ckmpm.mpm_ad_forward(ad.h, n - 1, n - 1, s1.data_ptr(), logE[1:].contiguous().data_ptr(),
                                     out1.data_ptr(), sc.dt, stream))
    ckmpm.check(ckmpm.mpm_ad_sync(ad.h, stream))
    got, want = _unpack(out[:, 1:].contiguous()), _unpack(out1)
    for k in ("x", "v", "B", "F"):
        assert nerr(got[k], want[k]) <= 1e-6, k
    ad.close()
    log("particle outside the domain: MPM_E_DOMAIN from forward and reverse call")


def _single_particle(sc, pos):
    """Scene sc cut down to its first particle, moved to `pos` on every axis."""
    import dataclasses
    x = np.full((1, 3), pos, np.float32)
    one = dataclasses.replace(sc, x=x, v=sc.v[:1].copy(), B=sc.B[:1].copy(), F=sc.F[:1].copy(), mat=sc.mat[:1].copy())
    one.logE = sc.logE[:1].copy()
    return one


def _gpu_rollout_grad(sc, nsteps, loss_name, target, F=None):
    import torch
    from paper_2412_10399_amd import diff
    ad = _ctx(sc)
    n = sc.n
    s0 = _state(sc, F=F)
    x0, B0, H0 = s0[0:3].t(), s0[6:15].t().reshape(n, 3, 3), s0[15:24].t().reshape(n, 3, 3)
    v0 = s0[3:6].t().clone().requires_grad_(True)
    logE = torch.from_numpy(sc.logE).cuda().requires_grad_(True)
    state0 = diff.planes(x0, v0, B0, H0)
    fin = diff.rollout(ad, state0, logE, nsteps, sc.dt, checkpoint_every=8)
    x = fin[0:3].t()
    com = x.mean(dim=0)
    if loss_name == "com":
        loss = ((com - torch.tensor(target, dtype=torch.float32, device="cuda")) ** 2).sum()
    else:
        loss = ((x - com) ** 2).sum(dim=1).mean()
    loss.backward()
    out = float(loss.detach()), v0.grad.double().cpu().numpy(), logE.grad.double().cpu().numpy()
    ad.close()
    return out


@pytest.mark.parametrize("loss_name", ["com", "spread"])
def test_rollout_gradient_matches_oracle_adjoint(loss_name):
    """The differentiation workload in full: 65,536 particles, 64 steps, checkpoints
    every 8 steps; gradients in v0 and log E against the FP64 oracle's adjoint
    (pinned itself by differences).  For the centre-of-mass loss the log E gradient
    vanishes (internal stress conserves momentum and no wall is reached); the GPU's
    is checked to be negligible against the scale of the v0 gradient times the
    per-step velocity change a modulus change can cause."""
    sc = scenes.diff_box()
    assert sc.n == 65536
    nsteps = sc.steps
    target = scenes.diff_target()
    loss, gv, gl = _gpu_rollout_grad(sc, nsteps, loss_name, target)
    cfg, mats = oracle.scene_config(sc), oracle.scene_materials(sc)
    st0 = oracle.State.from_scene(sc)
    ol = oracle.com_loss(target) if loss_name == "com" else oracle.spread_loss
    ref_loss, ref = oracle.rollout_loss_grad(cfg, mats, st0, sc.dt, nsteps, ol)
    ev = nerr(gv, ref["v"])
    log("%s loss %.6e (oracle %.6e), d/dv0 %.2e" % (loss_name, loss, ref_loss, ev))
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss) + 1e-12
    assert ev <= 1e-3
    if loss_name == "spread":
        el = nerr(gl, ref["logE"])
        log("spread d/dlogE %.2e (max |oracle| %.3e)" % (el, np.abs(ref["logE"]).max()))
        assert el <= 1e-3
    else:
        log("com d/dlogE max |gpu| %.3e, max |oracle| %.3e" % (np.abs(gl).max(), np.abs(ref["logE"]).max()))
        assert np.abs(gl).max() <= 1e-4 * np.abs(gv).max()


def test_rollout_directional_derivatives_match_differences():
    """32 seeded unit directions (16 in v0, 16 in log E) of the spread loss after 64
    steps of the reduced workload (prestrained so that stiffness matters): the GPU
    gradient's directional derivatives against FP64 central differences of the
    oracle's forward rollout."""
    sc = scenes.diff_box(scale=4)
    rng0 = np.random.default_rng(9)
    sc.F = (np.eye(3)[None] + 0.02 * rng0.standard_normal((sc.n, 3, 3))).astype(np.float32)
    nsteps = 64
    _, gv, gl = _gpu_rollout_grad(sc, nsteps, "spread", None)
    cfg, mats = oracle.scene_config(sc), oracle.scene_materials(sc)
    st0 = oracle.State.from_scene(sc)
    rng = np.random.default_rng(17)
    worst = 0.0
    for k in range(32):
        field = "v" if k < 16 else "logE"
        base = getattr(st0, field)
        d = rng.standard_normal(base.shape)
        d /= np.linalg.norm(d)
        h = 1e-3
        sp, sm = st0.copy(), st0.copy()
        setattr(sp, field, base + h * d)
        setattr(sm, field, base - h * d)
        fd = (oracle.rollout_loss(cfg, mats, sp, sc.dt, nsteps, oracle.spread_loss)
              - oracle.rollout_loss(cfg, mats, sm, sc.dt, nsteps, oracle.spread_loss)) / (2 * h)
        an = float(((gv if field == "v" else gl) * d).sum())
        rel = abs(an - fd) / abs(fd)
        worst = max(worst, rel)
        assert rel <= 1e-3, (k, field, an, fd)
    log("32 directional derivatives: worst relative error %.2e" % worst)
