"""Host-side logic of bench.py (no GPU): the one-GPU guard, the measured-traffic
lookup (used only while the kernel sources match the committed counter runs) and
the step's algorithmic byte model."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_lookup_follows_the_source_digest(tmp_path, monkeypatch):
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    t["source_digest"] = bench.source_digest()
    good = tmp_path / "traffic.json"
    good.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    k = t["kernels"]["p2g"]
    want = (k["fetch_kib"] * t["fetch_scale"] + k["write_kib"] * t["write_scale"]) * 1024.0
    assert abs(bench.measured_traffic("p2g", 1) - want) <= 1e-9 * want
    assert bench.measured_traffic("no_such_kernel", 1) is None
    t["source_digest"] = "0" * 16
    good.write_text(json.dumps(t))
    assert bench.measured_traffic("p2g", 1) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("p2g", 1) is None


def test_step_byte_model():
    # P2G reads x, v, B, F (96 B); G2P reads x, F (48 B) and writes x, v, B, F (96 B)
    assert bench.STEP_PARTICLE_BYTES == 96 + 48 + 96
    # per active block: clear 2 KiB, P2G flush 2 KiB, update reads 2 KiB and writes
    # 1.5 KiB, G2P reads 1.5 KiB
    assert bench.STEP_GRID_BLOCK_BYTES == 2048 + 2048 + 2048 + 1536 + 1536


def test_checker_timing_helpers():
    """The CPU-baseline leg: host description, and the checker timed at one and at
    two threads on a small scene; the checker's state after a step does not depend
    on its thread count (its scatter is serial), so both timings run the same work."""
    import numpy as np

    import oracle
    import scenes
    h = bench.host_cpu()
    assert h["logical_cpus"] >= 1 and h["usable_cpus"] >= 1
    sc = scenes.random_blob(3, n_cells=(16, 16, 16), lo_cells=(5.0, 5.0, 5.0), ext_cells=(4, 4, 4), F_scale=0.02)
    states = []
    for threads in (1, 2):
        rate, steps, sec = bench.time_oracle(sc, threads, 2, 30.0)
        assert steps == 2 and rate > 0 and sec > 0
        oracle.set_num_threads(threads)
        assert oracle.num_threads() == threads
        st = oracle.State.from_scene(sc)
        oracle.step(oracle.scene_config(sc), oracle.scene_materials(sc), st, sc.dt)
        states.append(st)
    for name in ("x", "v", "B", "F"):
        assert np.array_equal(getattr(states[0], name), getattr(states[1], name)), name
