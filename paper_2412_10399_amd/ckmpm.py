"""Thin ctypes binding of libckmpm.so (the C ABI declared in include/ckmpm.h).

Functions carry the C names and only marshal arguments: every step of the MPM
path runs in the HIP library.  PyTorch tensors provide device memory
(`data_ptr()`) and streams (`torch.cuda.Stream.cuda_stream`).  If the library is
not built this module raises on first use; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libckmpm.so")
_lib = None

(MPM_OK, MPM_E_INVALID, MPM_E_OOM, MPM_E_DOMAIN, MPM_E_CAPACITY, MPM_E_NONFINITE, MPM_E_HIP, MPM_E_STALE, MPM_E_CFL,
 MPM_E_SCRATCH) = range(10)
MPM_NOALLOC_SCRATCH_BYTES = 32 * 1024 * 1024
MPM_FIXED_COROTATED, MPM_DRUCKER_PRAGER = 0, 1
MPM_BC_NONE, MPM_BC_STICKY = 0, 1
MPM_TRANSFER_MLS, MPM_TRANSFER_APIC, MPM_TRANSFER_PIC = 0, 1, 2
MPM_FLAG_FUSED_G2P2G = 1
MPM_FLAG_QUADRATIC = 2
MPM_STATE_PLANES = 27
PHASES = ("sort", "p2g", "grid_update", "g2p", "g2p2g")

# plane offsets inside one state buffer
X0, V0, B0, F0, R0 = 0, 3, 6, 15, 24


class CkMpmError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        super().__init__("%s: %s (%d)" % (what, status_string(status), status))
        self.status = status


class mpm_config(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32 * 3), ("dx", ctypes.c_double), ("origin", ctypes.c_double * 3),
                ("gravity", ctypes.c_double * 3), ("bc", ctypes.c_int32), ("bc_band", ctypes.c_int32),
                ("max_particles", ctypes.c_int64), ("max_blocks", ctypes.c_int64), ("transfer", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("deterministic", ctypes.c_int32)]


class mpm_material(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("E", ctypes.c_float), ("nu", ctypes.c_float), ("rho", ctypes.c_float),
                ("vol0", ctypes.c_float), ("friction_deg", ctypes.c_float)]


class mpm_particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("stride", ctypes.c_int64), ("state", ctypes.c_void_p * 2),
                ("id", ctypes.c_void_p * 2), ("mat", ctypes.c_void_p * 2), ("current", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class mpm_stats(ctypes.Structure):
    _fields_ = [("n_particle_blocks", ctypes.c_int64), ("n_grid_blocks", ctypes.c_int64),
                ("max_block_particles", ctypes.c_int64), ("status_bits", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class mpm_server_config(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_int64), ("max_jobs", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32), ("flags", ctypes.c_int32)]


class mpm_job_desc(ctypes.Structure):
    _fields_ = [("cfg", mpm_config), ("mats", ctypes.POINTER(mpm_material)), ("n_mat", ctypes.c_int32),
                ("nsteps", ctypes.c_int32), ("n", ctypes.c_int64), ("state", ctypes.c_void_p),
                ("mat", ctypes.c_void_p), ("dt", ctypes.c_double), ("stream", ctypes.c_void_p)]


class mpm_job_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("steps_done", ctypes.c_int32), ("n", ctypes.c_int64),
                ("footprint", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


MPM_JOB_PENDING, MPM_JOB_ACTIVE, MPM_JOB_DONE, MPM_JOB_FAILED = range(4)
MPM_SERVER_GROUPED = 1

EXPORTS = ("mpm_create", "mpm_destroy", "mpm_p2g", "mpm_grid_update", "mpm_g2p", "mpm_step", "mpm_sync",
           "mpm_grid_read", "mpm_current_buffer", "mpm_sort_keys", "mpm_invalidate", "mpm_get_stats", "mpm_profile_enable",
           "mpm_profile_read", "mpm_status_string", "mpm_abi_version", "mpm_footprint", "mpm_server_create",
           "mpm_server_destroy", "mpm_server_submit", "mpm_server_poll", "mpm_server_drain", "mpm_server_job_info",
           "mpm_server_job_read", "mpm_server_job_release", "mpm_server_step_latencies", "mpm_ad_create",
           "mpm_ad_destroy", "mpm_ad_forward", "mpm_ad_backward", "mpm_ad_sync", "mpm_step_noalloc")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libckmpm.so is not built (expected at %s); run __graft_entry__.build()" % _LIB_PATH)
        L = ctypes.CDLL(_LIB_PATH)
        vp, st = ctypes.c_void_p, ctypes.c_int
        L.mpm_create.argtypes = [ctypes.POINTER(mpm_config), ctypes.POINTER(mpm_material), ctypes.c_int32,
                                 ctypes.POINTER(vp)]
        L.mpm_destroy.argtypes = [vp]
        L.mpm_p2g.argtypes = [vp, ctypes.POINTER(mpm_particles), ctypes.c_double, vp]
        L.mpm_grid_update.argtypes = [vp, ctypes.c_double, vp]
        L.mpm_g2p.argtypes = [vp, ctypes.POINTER(mpm_particles), ctypes.c_double, vp]
        L.mpm_step.argtypes = [vp, ctypes.POINTER(mpm_particles), ctypes.c_double, ctypes.c_int32, vp]
        L.mpm_step_noalloc.argtypes = [ctypes.POINTER(mpm_config), ctypes.POINTER(mpm_material), ctypes.c_int32,
                                       ctypes.POINTER(mpm_particles), ctypes.c_double, ctypes.c_int32, vp, vp]
        L.mpm_sync.argtypes = [vp, vp]
        L.mpm_grid_read.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
        L.mpm_current_buffer.argtypes = [vp]
        L.mpm_sort_keys.argtypes = [vp, ctypes.POINTER(mpm_particles), vp, vp, vp]
        L.mpm_invalidate.argtypes = [vp]
        L.mpm_get_stats.argtypes = [vp, ctypes.POINTER(mpm_stats), vp]
        L.mpm_profile_enable.argtypes = [vp, ctypes.c_int32]
        L.mpm_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.c_int32]
        L.mpm_status_string.argtypes = [st]
        L.mpm_status_string.restype = ctypes.c_char_p
        L.mpm_abi_version.restype = ctypes.c_int32
        L.mpm_footprint.argtypes = [ctypes.POINTER(mpm_config), ctypes.c_int64]
        L.mpm_footprint.restype = ctypes.c_int64
        i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
        L.mpm_server_create.argtypes = [ctypes.POINTER(mpm_server_config), ctypes.POINTER(vp)]
        L.mpm_server_destroy.argtypes = [vp]
        L.mpm_server_submit.argtypes = [vp, ctypes.POINTER(mpm_job_desc), i64p]
        L.mpm_server_poll.argtypes = [vp, i32p, i32p, i32p]
        L.mpm_server_drain.argtypes = [vp]
        L.mpm_server_job_info.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(mpm_job_info)]
        L.mpm_server_job_read.argtypes = [vp, ctypes.c_int64, vp, vp]
        L.mpm_server_job_release.argtypes = [vp, ctypes.c_int64]
        L.mpm_server_step_latencies.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int64, i64p]
        L.mpm_ad_create.argtypes = [ctypes.POINTER(mpm_config), ctypes.POINTER(mpm_material), ctypes.POINTER(vp)]
        L.mpm_ad_destroy.argtypes = [vp]
        L.mpm_ad_forward.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, vp, vp, vp, ctypes.c_double, vp]
        L.mpm_ad_backward.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.c_double, vp]
        L.mpm_ad_sync.argtypes = [vp, vp]
        for name in EXPORTS:
            if name not in ("mpm_status_string", "mpm_abi_version", "mpm_footprint", "mpm_current_buffer"):
                getattr(L, name).restype = st
        L.mpm_current_buffer.restype = ctypes.c_int32
        _lib = L
    return _lib


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


# ----------------------------------------------------------------- C ABI mirror
def mpm_create(cfg: mpm_config, mats: Sequence[mpm_material]):
    arr = (mpm_material * len(mats))(*mats)
    h = ctypes.c_void_p()
    s = lib().mpm_create(ctypes.byref(cfg), arr, len(mats), ctypes.byref(h))
    return s, h


def mpm_destroy(ctx) -> int:
    return lib().mpm_destroy(ctx)


def mpm_p2g(ctx, parts: mpm_particles, dt: float, stream=None) -> int:
    return lib().mpm_p2g(ctx, ctypes.byref(parts), float(dt), _stream(stream))


def mpm_grid_update(ctx, dt: float, stream=None) -> int:
    return lib().mpm_grid_update(ctx, float(dt), _stream(stream))


def mpm_g2p(ctx, parts: mpm_particles, dt: float, stream=None) -> int:
    return lib().mpm_g2p(ctx, ctypes.byref(parts), float(dt), _stream(stream))


def mpm_step(ctx, parts: mpm_particles, dt: float, nsteps: int, stream=None) -> int:
    return lib().mpm_step(ctx, ctypes.byref(parts), float(dt), int(nsteps), _stream(stream))


def mpm_step_noalloc(cfg: mpm_config, mats: Sequence[mpm_material], parts: mpm_particles, dt: float, nsteps: int,
                     status_ptr: Optional[int] = None, stream=None) -> int:
    """mpm_step without a context: library buffers from the static device scratch;
    status_ptr is a device int32 that receives the device-detected status (or None)."""
    arr = (mpm_material * len(mats))(*mats)
    return lib().mpm_step_noalloc(ctypes.byref(cfg), arr, len(mats), ctypes.byref(parts), float(dt), int(nsteps),
                                  status_ptr, _stream(stream))


def mpm_sync(ctx, stream=None) -> int:
    return lib().mpm_sync(ctx, _stream(stream))


def mpm_grid_read(ctx, grid: int, m_ptr: Optional[int], vec_ptr: Optional[int], stream=None) -> int:
    return lib().mpm_grid_read(ctx, int(grid), m_ptr, vec_ptr, _stream(stream))


def mpm_current_buffer(ctx) -> int:
    return int(lib().mpm_current_buffer(ctx))


def mpm_sort_keys(ctx, parts: mpm_particles, keys_ptr: Optional[int], perm_ptr: Optional[int], stream=None) -> int:
    return lib().mpm_sort_keys(ctx, ctypes.byref(parts), keys_ptr, perm_ptr, _stream(stream))


def mpm_invalidate(ctx) -> int:
    return lib().mpm_invalidate(ctx)


def mpm_get_stats(ctx, stream=None):
    out = mpm_stats()
    s = lib().mpm_get_stats(ctx, ctypes.byref(out), _stream(stream))
    return s, out


def mpm_profile_enable(ctx, enable: bool) -> int:
    return lib().mpm_profile_enable(ctx, 1 if enable else 0)


def mpm_profile_read(ctx, n_phases: int = 5):
    ms = (ctypes.c_double * n_phases)()
    cnt = (ctypes.c_int64 * n_phases)()
    s = lib().mpm_profile_read(ctx, ms, cnt, n_phases)
    return s, list(ms), list(cnt)


def mpm_ad_create(cfg: mpm_config, mat: mpm_material):
    h = ctypes.c_void_p()
    s = lib().mpm_ad_create(ctypes.byref(cfg), ctypes.byref(mat), ctypes.byref(h))
    return s, h


def mpm_ad_destroy(h) -> int:
    return lib().mpm_ad_destroy(h)


def mpm_ad_forward(h, n: int, stride: int, state_in: int, logE: int, state_out: int, dt: float, stream=None) -> int:
    return lib().mpm_ad_forward(h, n, stride, state_in, logE, state_out, dt, _stream(stream))


def mpm_ad_backward(h, n: int, stride: int, state_in: int, logE: int, cot_out: int, cot_in: int, logE_cot: int,
                    dt: float, stream=None) -> int:
    return lib().mpm_ad_backward(h, n, stride, state_in, logE, cot_out, cot_in, logE_cot, dt, _stream(stream))


def mpm_ad_sync(h, stream=None) -> int:
    return lib().mpm_ad_sync(h, _stream(stream))


def mpm_status_string(status: int) -> str:
    return lib().mpm_status_string(int(status)).decode()


def mpm_abi_version() -> int:
    return lib().mpm_abi_version()


def mpm_footprint(cfg: mpm_config, n: int) -> int:
    """Device bytes of a context with `cfg` plus two ping-pong buffers of n particles."""
    return int(lib().mpm_footprint(ctypes.byref(cfg), int(n)))


def mpm_server_create(cfg: mpm_server_config):
    h = ctypes.c_void_p()
    s = lib().mpm_server_create(ctypes.byref(cfg), ctypes.byref(h))
    return s, h


def mpm_server_destroy(srv) -> int:
    return lib().mpm_server_destroy(srv)


def mpm_server_submit(srv, desc: mpm_job_desc):
    jid = ctypes.c_int64(-1)
    s = lib().mpm_server_submit(srv, ctypes.byref(desc), ctypes.byref(jid))
    return s, jid.value


def mpm_server_poll(srv):
    p, a, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    s = lib().mpm_server_poll(srv, ctypes.byref(p), ctypes.byref(a), ctypes.byref(d))
    return s, p.value, a.value, d.value


def mpm_server_drain(srv) -> int:
    return lib().mpm_server_drain(srv)


def mpm_server_job_info(srv, job_id: int):
    out = mpm_job_info()
    s = lib().mpm_server_job_info(srv, int(job_id), ctypes.byref(out))
    return s, out


def mpm_server_job_read(srv, job_id: int, state_ptr: Optional[int], ids_ptr: Optional[int]) -> int:
    return lib().mpm_server_job_read(srv, int(job_id), state_ptr, ids_ptr)


def mpm_server_job_release(srv, job_id: int) -> int:
    return lib().mpm_server_job_release(srv, int(job_id))


def mpm_server_step_latencies(srv):
    count = ctypes.c_int64(0)
    s = lib().mpm_server_step_latencies(srv, None, 0, ctypes.byref(count))
    if s != MPM_OK or count.value == 0:
        return s, []
    buf = (ctypes.c_double * count.value)()
    s = lib().mpm_server_step_latencies(srv, buf, count.value, ctypes.byref(count))
    return s, list(buf)


def status_string(status: int) -> str:
    try:
        return mpm_status_string(status)
    except Exception:  # library missing: still format the error
        return "status"


def check(status: int, what: str = "ckmpm") -> None:
    if status != MPM_OK:
        raise CkMpmError(status, what)


# --------------------------------------------------------- struct construction
def make_config(n_cells, dx, origin=(0.0, 0.0, 0.0), gravity=(0.0, 0.0, 0.0), bc_band=0, max_particles=1,
                max_blocks=1024, bc=None, fused=False, quadratic=False, transfer=0,
                deterministic=False) -> mpm_config:
    c = mpm_config()
    for a in range(3):
        c.n_cells[a] = int(n_cells[a])
        c.origin[a] = float(origin[a])
        c.gravity[a] = float(gravity[a])
    c.dx = float(dx)
    c.bc = (MPM_BC_STICKY if bc_band > 0 else MPM_BC_NONE) if bc is None else int(bc)
    c.bc_band = int(bc_band)
    c.max_particles = int(max_particles)
    c.max_blocks = int(max_blocks)
    c.transfer = int(transfer)
    c.flags = (MPM_FLAG_FUSED_G2P2G if fused else 0) | (MPM_FLAG_QUADRATIC if quadratic else 0)
    c.deterministic = 1 if deterministic else 0
    return c


def make_material(model, E, nu, rho, vol0, friction_deg=30.0) -> mpm_material:
    m = mpm_material()
    m.model, m.E, m.nu, m.rho, m.vol0, m.friction_deg = int(model), E, nu, rho, vol0, friction_deg
    return m


def state_planes(x, v, B, F):
    """Host arrays (N,3), (N,3), (N,3,3), (N,3,3) as the (27, N) FP32 state layout;
    the deformation gradient is stored as H = F - I (formed in FP64, then rounded),
    the position as its FP32 rounding x and the FP32 remainder r of an FP64 x."""
    import numpy as np
    n = len(x)
    planes = np.zeros((MPM_STATE_PLANES, n), np.float32)
    x64 = np.asarray(x, np.float64).reshape(n, 3)
    xh = x64.astype(np.float32)
    planes[X0:X0 + 3] = xh.T
    planes[R0:R0 + 3] = (x64 - xh.astype(np.float64)).astype(np.float32).T
    planes[V0:V0 + 3] = np.asarray(v, np.float32).reshape(n, 3).T
    planes[B0:B0 + 9] = np.asarray(B, np.float32).reshape(n, 9).T
    H = np.asarray(F, np.float64).reshape(n, 3, 3) - np.eye(3)[None]
    planes[F0:F0 + 9] = H.reshape(n, 9).T.astype(np.float32)
    return planes


def unpack_state(planes, ids=None):
    """(27, N) state planes (host) as dict(x, x32, v, B, H, F[, id]): x = x32 + r and
    F = I + H formed in FP64, x32 the FP32 position plane as stored."""
    import numpy as np
    n = planes.shape[1]
    H = planes[F0:F0 + 9].T.reshape(n, 3, 3).copy()
    x32 = planes[X0:X0 + 3].T.copy()
    out = dict(x=x32.astype(np.float64) + planes[R0:R0 + 3].T.astype(np.float64), x32=x32,
               v=planes[V0:V0 + 3].T.copy(), B=planes[B0:B0 + 9].T.reshape(n, 3, 3).copy(), H=H,
               F=H.astype(np.float64) + np.eye(3)[None])
    if ids is not None:
        out["id"] = np.asarray(ids).copy()
    return out


class Particles:
    """Device particle storage: two ping-pong buffers of 27 FP32 planes, ids and
    optional material indices, as torch tensors on a GPU."""

    def __init__(self, n: int, stride: Optional[int] = None, device="cuda", with_mat: bool = False):
        import torch
        self.n = int(n)
        self.stride = int(stride if stride is not None else max(n, 1))
        self.state = torch.zeros((2, MPM_STATE_PLANES, self.stride), dtype=torch.float32, device=device)
        self.ids = torch.zeros((2, self.stride), dtype=torch.int32, device=device)
        self.mats = torch.zeros((2, self.stride), dtype=torch.uint8, device=device) if with_mat else None
        self.c = mpm_particles()
        self.c.n = self.n
        self.c.stride = self.stride
        for b in range(2):
            self.c.state[b] = self.state[b].data_ptr()
            self.c.id[b] = self.ids[b].data_ptr()
            self.c.mat[b] = self.mats[b].data_ptr() if with_mat else None
        self.c.current = 0

    @property
    def current(self) -> int:
        return int(self.c.current)

    def load(self, x, v, B, F, ids=None, mat=None):
        """Host arrays (N,3), (N,3), (N,3,3), (N,3,3) into the current buffer.  The
        deformation gradient is stored as H = F - I (formed in FP64, then rounded)."""
        import numpy as np
        import torch
        n = self.n
        planes = state_planes(x, v, B, F)
        cur = self.current
        self.state[cur, :, :n].copy_(torch.from_numpy(planes))
        idv = np.arange(n, dtype=np.int32) if ids is None else np.asarray(ids, np.int32)
        self.ids[cur, :n].copy_(torch.from_numpy(idv))
        if self.mats is not None:
            mv = np.zeros(n, np.uint8) if mat is None else np.asarray(mat, np.uint8)
            self.mats[cur, :n].copy_(torch.from_numpy(mv))

    def read(self):
        """Current buffer to host in storage (sorted) order: dict(x, x32, v, B, H, F, id[, mat]);
        x = x32 + r formed in FP64, H = F - I as stored (FP32), F = I + H formed in FP64."""
        cur = self.current
        n = self.n
        out = unpack_state(self.state[cur, :, :n].cpu().numpy(), self.ids[cur, :n].cpu().numpy())
        if self.mats is not None:
            out["mat"] = self.mats[cur, :n].cpu().numpy().copy()
        return out

    def read_by_id(self):
        """Current state reordered so that row k holds particle id k."""
        d = self.read()
        order = d["id"].argsort(kind="stable")
        return {k: v[order] for k, v in d.items()}


class Context:
    """RAII holder for an mpm_ctx handle."""

    def __init__(self, cfg: mpm_config, mats: Sequence[mpm_material]):
        s, h = mpm_create(cfg, mats)
        check(s, "mpm_create")
        self.h = h
        self.cfg = cfg

    def close(self):
        if self.h is not None and self.h.value:
            mpm_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def scene_config(sc, max_particles=None, max_blocks=None, fused=False, quadratic=False, transfer=0,
                 deterministic=False) -> mpm_config:
    """mpm_config for a scene from the `scenes` package."""
    n = sc.n if max_particles is None else max_particles
    if max_blocks is None:
        nb = 1
        for a in range(3):
            nb *= sc.n_cells[a] // 4 + 1
        max_blocks = min(nb, 2 * (n // 256) + 4096)
    return make_config(sc.n_cells, sc.dx, sc.origin, sc.gravity, sc.bc_band, max(n, 1), max_blocks, fused=fused,
                       quadratic=quadratic, transfer=transfer, deterministic=deterministic)


def scene_materials(sc):
    return [make_material(m.model, m.E, m.nu, m.rho, m.vol0, m.friction_deg) for m in sc.materials]


def particles_from_scene(sc, device="cuda") -> Particles:
    p = Particles(sc.n, device=device, with_mat=len(sc.materials) > 1)
    p.load(sc.x, sc.v, sc.B, sc.F, mat=sc.mat)
    return p


def job_config(sc, margin_blocks: int = 3, fused=False, deterministic=False) -> mpm_config:
    """mpm_config for a served job: capacities sized to the scene's extent (blocks
    of the particles' bounding box grown by a margin on every side, twice over for
    the two grids) rather than to the whole grid."""
    import numpy as np
    lo = np.floor(sc.x.min(axis=0) / sc.dx).astype(np.int64)
    hi = np.floor(sc.x.max(axis=0) / sc.dx).astype(np.int64)
    nb = 1
    for a in range(3):
        nb *= int((hi[a] - lo[a]) // 4 + 2 + 2 * margin_blocks)
    return scene_config(sc, max_particles=sc.n, max_blocks=2 * nb + 64, fused=fused, deterministic=deterministic)


class Server:
    """RAII holder for an mpm_server handle, with torch-owned job inputs kept alive
    until the job is released."""

    def __init__(self, memory_budget: int, max_jobs: int = 32, n_streams: int = 4, steps_per_launch: int = 8,
                 grouped: bool = False):
        cfg = mpm_server_config()
        cfg.memory_budget = int(memory_budget)
        cfg.max_jobs = int(max_jobs)
        cfg.n_streams = int(n_streams)
        cfg.steps_per_launch = int(steps_per_launch)
        cfg.flags = MPM_SERVER_GROUPED if grouped else 0
        s, h = mpm_server_create(cfg)
        check(s, "mpm_server_create")
        self.h = h
        self._inputs = {}

    def submit(self, cfg: mpm_config, mats: Sequence[mpm_material], state, nsteps: int, dt: float, mat=None) -> int:
        """Queue a job; `state` is a (27, n) float32 CUDA tensor (`state_planes` layout), `mat` an
        optional (n,) uint8 CUDA tensor."""
        arr = (mpm_material * len(mats))(*mats)
        d = mpm_job_desc()
        d.cfg = cfg
        d.mats = arr
        d.n_mat = len(mats)
        d.nsteps = int(nsteps)
        d.n = int(state.shape[1])
        d.state = state.data_ptr()
        d.mat = mat.data_ptr() if mat is not None else None
        d.dt = float(dt)
        # the admission copy waits for the work torch queued on its current stream,
        # which produced `state` and `mat`
        import torch
        d.stream = _stream(torch.cuda.current_stream())
        s, jid = mpm_server_submit(self.h, d)
        check(s, "mpm_server_submit")
        self._inputs[jid] = (state, mat)
        return jid

    def submit_scene(self, sc, nsteps: int, device="cuda", deterministic=False) -> int:
        import torch
        state = torch.from_numpy(state_planes(sc.x, sc.v, sc.B, sc.F)).to(device)
        mat = torch.from_numpy(sc.mat.astype("uint8")).to(device) if len(sc.materials) > 1 else None
        return self.submit(job_config(sc, deterministic=deterministic), scene_materials(sc), state, nsteps, sc.dt, mat)

    def poll(self):
        s, p, a, d = mpm_server_poll(self.h)
        check(s, "mpm_server_poll")
        return p, a, d

    def drain(self):
        check(mpm_server_drain(self.h), "mpm_server_drain")

    def info(self, jid: int) -> mpm_job_info:
        s, out = mpm_server_job_info(self.h, jid)
        check(s, "mpm_server_job_info")
        return out

    def read(self, jid: int):
        """Final state of a finished job, reordered so that row k holds particle k."""
        import torch
        n = int(self.info(jid).n)
        st = torch.empty((MPM_STATE_PLANES, n), dtype=torch.float32, device="cuda")
        ids = torch.empty(n, dtype=torch.int32, device="cuda")
        check(mpm_server_job_read(self.h, jid, st.data_ptr(), ids.data_ptr()), "mpm_server_job_read")
        d = unpack_state(st.cpu().numpy(), ids.cpu().numpy())
        order = d["id"].argsort(kind="stable")
        return {k: v[order] for k, v in d.items()}

    def release(self, jid: int):
        check(mpm_server_job_release(self.h, jid), "mpm_server_job_release")
        self._inputs.pop(jid, None)

    def step_latencies(self):
        s, lat = mpm_server_step_latencies(self.h)
        check(s, "mpm_server_step_latencies")
        return lat

    def close(self):
        if self.h is not None and self.h.value:
            mpm_server_destroy(self.h)
        self.h = None
        self._inputs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
