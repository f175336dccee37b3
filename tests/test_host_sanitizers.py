"""Host code under AddressSanitizer (and UndefinedBehaviorSanitizer for the checker),
on the CPU: the FP64 checker's entry points on a small scene, and the HIP library's
host-side paths that need no GPU (validation of configurations and arguments,
status strings, footprints, the no-allocation step's size check).  Each driver is
built in a temporary directory; a sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/lib/llvm/bin/clang"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ORACLE_DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include "ckmpm_oracle.h"

static unsigned long long lcg = 12345;
static double unif() { lcg = lcg * 6364136223846793005ull + 1442695040888963407ull; return (lcg >> 11) * (1.0 / 9007199254740992.0); }

int main() {
    ora_config cfg{};
    for (int a = 0; a < 3; ++a) cfg.n_cells[a] = 12;
    cfg.dx = 1.0 / 16;
    cfg.gravity[1] = -9.8;
    cfg.bc_band = 2;
    ora_material mats[2] = {{0, 1e4, 0.3, 1000.0, cfg.dx * cfg.dx * cfg.dx / 8, 30.0},
                            {1, 3.5e5, 0.3, 1600.0, cfg.dx * cfg.dx * cfg.dx / 8, 30.0}};
    const int n = 4 * 4 * 4 * 8;
    std::vector<double> x(3 * n), v(3 * n), B(9 * n), F(9 * n);
    std::vector<uint8_t> mat(n);
    for (int p = 0; p < n; ++p) {
        const int c = p / 8, s = p % 8;
        const int cc[3] = {c % 4, (c / 4) % 4, c / 16};
        for (int a = 0; a < 3; ++a) {
            x[3 * p + a] = (4.0 + cc[a] + 0.5 * ((s >> a) & 1) + 0.5 * unif()) * cfg.dx;
            v[3 * p + a] = 0.2 * (unif() - 0.5);
        }
        for (int i = 0; i < 9; ++i) {
            B[9 * p + i] = 1e-4 * (unif() - 0.5);
            F[9 * p + i] = (i % 4 == 0 ? 1.0 : 0.0) + 0.02 * (unif() - 0.5);
        }
        mat[p] = (uint8_t)(p & 1);
    }
    const int64_t nodes = 2 * 13 * 13 * 13;
    std::vector<double> gm(nodes), gp(3 * nodes), gv(3 * nodes), diag(32);
    ora_outputs out{gm.data(), gp.data(), gv.data(), diag.data()};
    int bad = 0;
    for (int t = 0; t < 3; ++t) {
        cfg.transfer = t;
        std::vector<double> x1 = x, v1 = v, B1 = B, F1 = F;
        for (int k = 0; k < 2; ++k)
            bad |= ora_step(&cfg, mats, 2, n, x1.data(), v1.data(), B1.data(), F1.data(), mat.data(), nullptr, 1e-4, &out);
    }
    cfg.transfer = 0;
    {
        std::vector<double> x1 = x, v1 = v, B1 = B, F1 = F;
        bad |= ora_step_quadratic(&cfg, mats, 2, n, x1.data(), v1.data(), B1.data(), F1.data(), mat.data(), nullptr,
                                  1e-4, &out);
    }
    {
        std::vector<double> logE(n, std::log(1e4)), xb(3 * n, 1.0), vb(3 * n, 0.5), Bb(9 * n, 0.1), Fb(9 * n, 0.2);
        std::vector<double> xo(3 * n), vo(3 * n), Bo(9 * n), Fo(9 * n), lo(n);
        std::vector<uint8_t> zero(n, 0);
        bad |= ora_step_vjp(&cfg, mats, 1, n, x.data(), v.data(), B.data(), F.data(), zero.data(), logE.data(), 1e-4,
                            xb.data(), vb.data(), Bb.data(), Fb.data(), xo.data(), vo.data(), Bo.data(), Fo.data(),
                            lo.data());
    }
    std::vector<float> xs(3 * n);
    for (int p = 0; p < n; ++p)
        for (int a = 0; a < 3; ++a) xs[a * n + p] = (float)x[3 * p + a];
    std::vector<uint32_t> keys(n), perm(n);
    int32_t nb = 0;
    ora_cell_keys(&cfg, n, xs.data(), n, keys.data(), &nb);
    ora_stable_sort(n, keys.data(), perm.data());
    double U[9], S[3], V[9], tau[9];
    bad |= ora_svd3(F.data(), U, S, V) < 0;
    ora_kirchhoff(&mats[0], NAN, F.data(), tau);
    std::printf("checker %s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
"""

LIB_DRIVER = r"""
#include <stdio.h>
#include <string.h>
#include "ckmpm.h"
int main(void) {
    int bad = 0;
    if (mpm_abi_version() != CKMPM_ABI_VERSION) bad |= 1;
    for (int s = 0; s <= 10; ++s)
        if (!mpm_status_string((mpm_status)s)) bad |= 2;
    mpm_config c;
    memset(&c, 0, sizeof c);
    c.n_cells[0] = c.n_cells[1] = c.n_cells[2] = 32;
    c.dx = 1.0 / 32;
    c.max_particles = 1000;
    c.max_blocks = 100;
    mpm_material m;
    memset(&m, 0, sizeof m);
    m.model = 0; m.E = 1e4f; m.nu = 0.3f; m.rho = 1000.f; m.vol0 = 1e-5f;
    if (mpm_footprint(&c, 1000) <= 0) bad |= 4;
    mpm_ctx *ctx = 0;
    c.dx = 0.03;
    if (mpm_create(&c, &m, 1, &ctx) != MPM_E_INVALID || ctx) bad |= 8;
    c.dx = 1.0 / 32;
    m.nu = 0.5f;
    if (mpm_create(&c, &m, 1, &ctx) != MPM_E_INVALID) bad |= 16;
    m.nu = 0.3f;
    c.max_particles = 1 << 22;
    mpm_particles p;
    memset(&p, 0, sizeof p);
    if (mpm_step_noalloc(&c, &m, 1, &p, 1e-3, 1, 0, 0) != MPM_E_SCRATCH) bad |= 32;
    if (mpm_step(0, &p, 1e-3, 1, 0) != MPM_E_INVALID) bad |= 64;
    if (mpm_destroy(0) != MPM_OK) bad |= 128;
    if (mpm_current_buffer(0) != -1) bad |= 256;
    mpm_server_config sc;
    memset(&sc, 0, sizeof sc);
    mpm_server *srv = 0;
    if (mpm_server_create(&sc, &srv) != MPM_E_INVALID) bad |= 512;
    printf("library host paths %s (%d)\n", bad ? "FAILED" : "ok", bad);
    return bad;
}
"""


def _run(cmd, env=None, cwd=None):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=cwd)
    return r.returncode, r.stdout + r.stderr


def _clean(out):
    return "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out


def test_checker_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    (tmp_path / "drv.cpp").write_text(ORACLE_DRIVER)
    exe = tmp_path / "drv"
    rc, out = _run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"), str(tmp_path / "drv.cpp"),
                    os.path.join(ROOT, "oracle", "ckmpm_oracle.cpp"), "-o", str(exe)])
    assert rc == 0, out[-3000:]
    rc, out = _run([str(exe)])
    assert rc == 0 and _clean(out) and "checker ok" in out, out[-3000:]


def test_library_host_paths_under_address_sanitizer(tmp_path):
    if not (os.path.exists(CLANG) and os.path.exists(HIPCC)):
        pytest.skip("no ROCm toolchain")
    lib = tmp_path / "libckmpm_asan.so"
    srcs = sorted(os.path.join(ROOT, "paper_2412_10399_amd", "csrc", f)
                  for f in os.listdir(os.path.join(ROOT, "paper_2412_10399_amd", "csrc")) if f.endswith(".hip"))
    # the sanitizer instruments host code only
    rc, out = _run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared", "-munsafe-fp-atomics",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), "-o", str(lib)] + srcs)
    assert rc == 0, out[-3000:]
    (tmp_path / "drv.c").write_text(LIB_DRIVER)
    exe = tmp_path / "drv"
    rc, out = _run([CLANG, "-fsanitize=address", "-I", os.path.join(ROOT, "include"), str(tmp_path / "drv.c"),
                    "-L", str(tmp_path), "-lckmpm_asan", "-Wl,-rpath," + str(tmp_path), "-o", str(exe)])
    assert rc == 0, out[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    rc, out = _run([str(exe)], env=env)
    assert rc == 0 and _clean(out) and "library host paths ok" in out, out[-3000:]
