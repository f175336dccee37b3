"""The numerical-diffusion diagnostic on the GPU: kinetic and elastic energy of the
high-frequency cuboid after five steps with the compact kernel and with the
quadratic B-spline kernel, against the oracle's FP64 steps of the same scene
(shortened 7-fold along z)."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_util import GpuRun, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("quadratic", [False, True])
def test_energy_after_five_steps_matches_oracle(quadratic):
    from paper_2412_10399_amd import diagnostics
    sc = scenes.diffusion_cuboid(scale=7)
    m = sc.materials[0]
    run = GpuRun(sc, quadratic=quadratic)
    got = run.steps(sc.dt, 5)
    run.close()
    assert got["status"] == 0
    k, e = diagnostics.energies(got["v"], got["F"], m.rho * m.vol0, m.vol0, m.E, m.nu)
    st = oracle.State.from_scene(sc)
    cfg, mats = oracle.scene_config(sc), oracle.scene_materials(sc)
    for _ in range(5):
        status, _, _ = (oracle.step_quadratic if quadratic else oracle.step)(cfg, mats, st, sc.dt)
        assert status == 0
    kr, er = diagnostics.energies(st.v, st.F, m.rho * m.vol0, m.vol0, m.E, m.nu)
    log("%s: kinetic %.6e (oracle %.6e), elastic %.6e (oracle %.6e)" % ("quadratic" if quadratic else "compact",
                                                                     k, kr, e, er))
    assert abs(k - kr) <= 1e-5 * kr
    assert abs(e - er) <= 1e-4 * er
