"""CPU-side checks of the C ABI: the built library loads and exports every entry
point include/*.h declares, struct layouts match the header, and host-side
validation rejects bad configurations before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ckmpm.h")
LIB = os.path.join(ROOT, "paper_2412_10399_amd", "libckmpm.so")


@pytest.fixture(scope="module")
def ck():
    if not os.path.exists(LIB):
        from paper_2412_10399_amd import build
        build.build()
    from paper_2412_10399_amd import ckmpm
    ckmpm.lib()
    return ckmpm


def declared_functions():
    import glob
    text = "".join(open(h).read() for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
    return sorted(set(re.findall(r"^\s*(?:mpm_status|const char \*|int32_t|int64_t)\s*\*?\s*(mpm_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported(ck):
    names = declared_functions()
    assert len(names) >= 15
    L = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ck.EXPORTS)


def test_abi_version_and_strings(ck):
    assert ck.mpm_abi_version() == 3
    for s in range(10):
        assert len(ck.mpm_status_string(s)) >= 2
    assert ck.mpm_status_string(10) == "unknown status"


def test_struct_layouts(ck):
    # sizes implied by the C declarations (natural alignment, x86-64)
    assert ctypes.sizeof(ck.mpm_config) == 4 * 3 + 4 + 8 + 24 + 24 + 4 + 4 + 8 + 8 + 4 + 4 + 4 + 4
    assert ck.mpm_config.deterministic.offset == 104
    assert ctypes.sizeof(ck.mpm_material) == 24
    assert ctypes.sizeof(ck.mpm_particles) == 8 + 8 + 16 + 16 + 16 + 4 + 4
    assert ctypes.sizeof(ck.mpm_stats) == 32


def _good():
    from paper_2412_10399_amd import ckmpm
    cfg = ckmpm.make_config((32, 32, 32), 1 / 32, max_particles=1000, max_blocks=100)
    mat = ckmpm.make_material(0, 1e4, 0.3, 1000.0, 1e-5)
    return cfg, mat


@pytest.mark.parametrize("field,value", [
    ("dx", 0.03), ("dx", -0.5), ("dx", 0.0), ("max_particles", 0), ("max_particles", 1 << 26),
    ("max_blocks", 0), ("bc", 7), ("bc_band", -1), ("transfer", 3), ("transfer", -1), ("flags", 3), ("flags", 4), ("flags", -1),
    ("deterministic", 2), ("deterministic", -1),
])
def test_invalid_config_rejected_on_host(ck, field, value):
    cfg, mat = _good()
    setattr(cfg, field, value)
    s, h = ck.mpm_create(cfg, [mat])
    assert s == ck.MPM_E_INVALID and not h.value


@pytest.mark.parametrize("flags,transfer", [(1, 0), (2, 0), (0, 1), (0, 2)])
def test_deterministic_mode_needs_plain_compact_mls(ck, flags, transfer):
    # the bitwise mode covers the phase kernels of the compact kernel with the MLS
    # transfer; every other combination is refused on the host
    cfg, mat = _good()
    cfg.deterministic = 1
    cfg.flags = flags
    cfg.transfer = transfer
    s, h = ck.mpm_create(cfg, [mat])
    assert s == ck.MPM_E_INVALID and not h.value


def test_footprint_counts_the_deterministic_staging(ck):
    cfg, _ = _good()
    plain = ck.mpm_footprint(cfg, 1000)
    cfg.deterministic = 1
    # 4 channels x 341 tile nodes x 4 bytes per block of max_blocks, padded like every buffer
    extra = (cfg.max_blocks * 4 * 341 * 4 + 256 + 255) // 256 * 256
    assert ck.mpm_footprint(cfg, 1000) - plain == extra


def test_current_buffer_of_null_context(ck):
    assert ck.mpm_current_buffer(None) == -1


@pytest.mark.parametrize("field,value", [("E", 0.0), ("nu", 0.5), ("nu", -0.1), ("rho", 0.0), ("vol0", -1.0),
                                         ("model", 5)])
def test_invalid_material_rejected_on_host(ck, field, value):
    cfg, mat = _good()
    setattr(mat, field, value)
    s, h = ck.mpm_create(cfg, [mat])
    assert s == ck.MPM_E_INVALID


def test_grid_too_large_and_bad_cells_rejected(ck):
    cfg, mat = _good()
    cfg.n_cells[0] = 2
    assert ck.mpm_create(cfg, [mat])[0] == ck.MPM_E_INVALID
    cfg, mat = _good()
    for a in range(3):
        cfg.n_cells[a] = 1 << 14   # (4097)^3 virtual blocks: keys would not fit 32 bits
    assert ck.mpm_create(cfg, [mat])[0] == ck.MPM_E_INVALID
    assert ck.lib().mpm_create(None, None, 1, None) == ck.MPM_E_INVALID
    assert ck.mpm_create(cfg, [])[0] == ck.MPM_E_INVALID


def test_calls_with_null_context_are_rejected(ck):
    p = ck.mpm_particles()
    assert ck.lib().mpm_p2g(None, ctypes.byref(p), 1e-3, None) == ck.MPM_E_INVALID
    assert ck.lib().mpm_grid_update(None, 1e-3, None) == ck.MPM_E_INVALID
    assert ck.lib().mpm_g2p(None, ctypes.byref(p), 1e-3, None) == ck.MPM_E_INVALID
    assert ck.lib().mpm_step(None, ctypes.byref(p), 1e-3, 1, None) == ck.MPM_E_INVALID
    assert ck.lib().mpm_sync(None, None) == ck.MPM_E_INVALID
    assert ck.mpm_destroy(None) == ck.MPM_OK


def test_product_path_has_no_checker_import():
    """The product package must not reach the CPU checker or any fallback."""
    pkg = os.path.join(ROOT, "paper_2412_10399_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f
                assert "import scenes" not in text, f


def test_struct_layouts_match_c_compiler(ck, tmp_path):
    """sizeof/offsetof from a C compiler reading include/ckmpm.h equal the ctypes mirror."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "ckmpm.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(mpm_config), sizeof(mpm_material), sizeof(mpm_particles), sizeof(mpm_stats));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(mpm_config, dx), offsetof(mpm_config, max_particles),
         offsetof(mpm_config, transfer), offsetof(mpm_particles, state), offsetof(mpm_particles, current));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(mpm_config, deterministic), sizeof(mpm_job_desc),
         offsetof(mpm_job_desc, dt), offsetof(mpm_job_desc, stream), sizeof(mpm_job_info));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    sizes = [int(v) for v in out[:4]]
    offs = [int(v) for v in out[4:9]]
    more = [int(v) for v in out[9:]]
    assert more == [ck.mpm_config.deterministic.offset, ctypes.sizeof(ck.mpm_job_desc), ck.mpm_job_desc.dt.offset,
                    ck.mpm_job_desc.stream.offset, ctypes.sizeof(ck.mpm_job_info)]
    assert sizes == [ctypes.sizeof(ck.mpm_config), ctypes.sizeof(ck.mpm_material), ctypes.sizeof(ck.mpm_particles),
                     ctypes.sizeof(ck.mpm_stats)]
    assert offs == [ck.mpm_config.dx.offset, ck.mpm_config.max_particles.offset, ck.mpm_config.transfer.offset,
                    ck.mpm_particles.state.offset, ck.mpm_particles.current.offset]


def test_noalloc_step_rejects_oversized_buffers_on_host(ck):
    """mpm_step_noalloc refuses, before any GPU work, a configuration whose buffers
    exceed its static scratch, and a bad configuration as mpm_create does."""
    cfg, mat = _good()
    cfg.max_particles = 1 << 22   # 34 B of sort scratch and stress per particle: 136 MiB
    p = ck.mpm_particles()
    L = ck.lib()
    assert L.mpm_step_noalloc(ctypes.byref(cfg), ctypes.byref(mat), 1, ctypes.byref(p), 1e-3, 1, None,
                              None) == ck.MPM_E_SCRATCH
    cfg, mat = _good()
    cfg.dx = 0.03
    assert L.mpm_step_noalloc(ctypes.byref(cfg), ctypes.byref(mat), 1, ctypes.byref(p), 1e-3, 1, None,
                              None) == ck.MPM_E_INVALID
    assert L.mpm_step_noalloc(None, None, 1, None, 1e-3, 1, None, None) == ck.MPM_E_INVALID


def test_footprint_per_grid_block(ck):
    # Per block of max_blocks: the bucket (2048 ids, 4 B) and its sub-cell codes (2 B),
    # the particle-block list, kept-order range (2), start and count, the two
    # grid-block lists, the two grids (512 floats each) and the kept neighbourhood
    # (27 pool-block indices).  With max_blocks a multiple of 64 every such buffer is
    # a whole number of 256-byte units, so the padding cancels in the difference.
    per_block = 2048 * 4 + 2048 * 2 + 4 + 2 * 4 + 4 + 4 + 2 * 4 + 2 * 512 * 4 + 27 * 4
    a = ck.make_config((32, 32, 32), 1 / 32, max_particles=1000, max_blocks=64)
    b = ck.make_config((32, 32, 32), 1 / 32, max_particles=1000, max_blocks=128)
    assert ck.mpm_footprint(b, 1000) - ck.mpm_footprint(a, 1000) == 64 * per_block


def test_adjoint_config_is_dense_while_affordable(ck):
    """diff.ad_config gives every lattice block a slot (dense grids, no marking) up to
    the memory budget, and the main step's pool size beyond it."""
    import scenes
    from paper_2412_10399_amd import diff
    sc = scenes.diff_box()
    nb = 17 ** 3
    assert diff.ad_config(sc).max_blocks == nb
    assert ck.scene_config(sc).max_blocks < nb          # the main step's pool would not cover it
    assert diff.ad_config(sc, direct_budget_mib=1).max_blocks == ck.scene_config(sc).max_blocks
