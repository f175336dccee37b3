"""FP64 CPU oracle for the compact-kernel MPM step (CK-MPM, arXiv 2412.10399).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the HIP library and
its Python binding) never touches it, and the two share no code.

Two independent implementations live here:
  * `ckmpm_oracle.cpp` (loaded through ctypes below): plain FP64 loops following
    the paper's step order, used at every size;
  * `bruteforce.py`: a numpy transcription at the level of the definitions
    (weights of every node of both grids, LAPACK SVD), used on tiny scenes to pin
    the C++ oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckmpm_oracle.cpp")
_LIB = os.path.join(_HERE, "libckmpm_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C++ oracle with g++ (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class OraConfig(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32 * 3), ("dx", ctypes.c_double), ("origin", ctypes.c_double * 3),
                ("gravity", ctypes.c_double * 3), ("bc_band", ctypes.c_int32), ("transfer", ctypes.c_int32)]


class OraMaterial(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("E", ctypes.c_double), ("nu", ctypes.c_double),
                ("rho", ctypes.c_double), ("vol0", ctypes.c_double), ("friction_deg", ctypes.c_double)]


class OraOutputs(ctypes.Structure):
    _fields_ = [("grid_m", ctypes.c_void_p), ("grid_p", ctypes.c_void_p), ("grid_v", ctypes.c_void_p),
                ("diag", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.ora_K1.restype = ctypes.c_double
        L.ora_K1.argtypes = [ctypes.c_double]
        L.ora_dK1.restype = ctypes.c_double
        L.ora_dK1.argtypes = [ctypes.c_double]
        L.ora_d2K1.restype = ctypes.c_double
        L.ora_d2K1.argtypes = [ctypes.c_double]
        L.ora_stencil.argtypes = [ctypes.POINTER(OraConfig), dp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.ora_moment_matrix.argtypes = [ctypes.POINTER(OraConfig), dp, dp]
        L.ora_svd3.argtypes = [dp, dp, dp, dp]
        L.ora_kirchhoff.argtypes = [ctypes.POINTER(OraMaterial), ctypes.c_double, dp, dp]
        L.ora_energy_density.restype = ctypes.c_double
        L.ora_energy_density.argtypes = [ctypes.POINTER(OraMaterial), ctypes.c_double, dp]
        L.ora_dp_return_map.argtypes = [ctypes.POINTER(OraMaterial), ctypes.c_double, dp]
        L.ora_kirchhoff_vjp.argtypes = [ctypes.POINTER(OraMaterial), ctypes.c_double, dp, dp, dp,
                                        ctypes.POINTER(ctypes.c_double)]
        L.ora_cell_keys.argtypes = [ctypes.POINTER(OraConfig), ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]
        L.ora_stable_sort.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        L.ora_step.restype = ctypes.c_int
        L.ora_step.argtypes = [ctypes.POINTER(OraConfig), ctypes.POINTER(OraMaterial), ctypes.c_int32,
                               ctypes.c_int64, dp, dp, dp, dp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                               ctypes.POINTER(OraOutputs)]
        L.ora_step_vjp.restype = ctypes.c_int
        L.ora_step_vjp.argtypes = [ctypes.POINTER(OraConfig), ctypes.POINTER(OraMaterial), ctypes.c_int32,
                                   ctypes.c_int64, dp, dp, dp, dp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                   dp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_void_p]
        L.ora_step_quadratic.restype = ctypes.c_int
        L.ora_step_quadratic.argtypes = L.ora_step.argtypes
        L.ora_Nq.restype = ctypes.c_double
        L.ora_Nq.argtypes = [ctypes.c_double]
        L.ora_dNq.restype = ctypes.c_double
        L.ora_dNq.argtypes = [ctypes.c_double]
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def config(n_cells, dx, origin=(0.0, 0.0, 0.0), gravity=(0.0, 0.0, 0.0), bc_band=0, transfer=0) -> OraConfig:
    c = OraConfig()
    for a in range(3):
        c.n_cells[a] = int(n_cells[a])
        c.origin[a] = float(origin[a])
        c.gravity[a] = float(gravity[a])
    c.dx = float(dx)
    c.bc_band = int(bc_band)
    c.transfer = int(transfer)
    return c


def material(model, E, nu, rho, vol0, friction_deg=30.0) -> OraMaterial:
    m = OraMaterial()
    m.model, m.E, m.nu, m.rho, m.vol0, m.friction_deg = int(model), E, nu, rho, vol0, friction_deg
    return m


def scene_config(sc, transfer=0) -> OraConfig:
    return config(sc.n_cells, sc.dx, sc.origin, sc.gravity, sc.bc_band, transfer)


def scene_materials(sc):
    arr = (OraMaterial * len(sc.materials))()
    for i, m in enumerate(sc.materials):
        arr[i] = material(m.model, m.E, m.nu, m.rho, m.vol0, m.friction_deg)
    return arr


def K1(x: float) -> float:
    return lib().ora_K1(float(x))


def dK1(x: float) -> float:
    return lib().ora_dK1(float(x))


def d2K1(x: float) -> float:
    return lib().ora_d2K1(float(x))


def stencil(cfg: OraConfig, xp):
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    nodes = np.zeros((2, 8, 3), np.int32)
    w = np.zeros((2, 8), np.float64)
    d = np.zeros((2, 8, 3), np.float64)
    lib().ora_stencil(ctypes.byref(cfg), _dptr(xp), nodes.ctypes.data, w.ctypes.data, d.ctypes.data)
    return nodes, w, d


def moment_matrix(cfg: OraConfig, xp) -> np.ndarray:
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    D = np.zeros((3, 3), np.float64)
    lib().ora_moment_matrix(ctypes.byref(cfg), _dptr(xp), _dptr(D))
    return D


def svd3(F):
    F = np.ascontiguousarray(F, dtype=np.float64)
    U = np.zeros((3, 3))
    S = np.zeros(3)
    V = np.zeros((3, 3))
    lib().ora_svd3(_dptr(F), _dptr(U), _dptr(S), _dptr(V))
    return U, S, V


def kirchhoff(mat: OraMaterial, F, logE: Optional[float] = None) -> np.ndarray:
    F = np.ascontiguousarray(F, dtype=np.float64)
    tau = np.zeros((3, 3))
    lib().ora_kirchhoff(ctypes.byref(mat), float("nan") if logE is None else float(logE), _dptr(F), _dptr(tau))
    return tau


def energy_density(mat: OraMaterial, F, logE: Optional[float] = None) -> float:
    F = np.ascontiguousarray(F, dtype=np.float64)
    return lib().ora_energy_density(ctypes.byref(mat), float("nan") if logE is None else float(logE), _dptr(F))


def kirchhoff_vjp(mat: OraMaterial, F, logE, tb):
    """Adjoint of the fixed-corotated Kirchhoff stress: (dL/dF, dL/dlogE) from dL/dtau."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    tb = np.ascontiguousarray(tb, dtype=np.float64)
    Fb = np.zeros((3, 3))
    lb = ctypes.c_double(0.0)
    lib().ora_kirchhoff_vjp(ctypes.byref(mat), float(logE), _dptr(F), _dptr(tb), _dptr(Fb), ctypes.byref(lb))
    return Fb, lb.value


def dp_return_map(mat: OraMaterial, F, logE: Optional[float] = None) -> np.ndarray:
    F = np.array(F, dtype=np.float64, order="C")
    lib().ora_dp_return_map(ctypes.byref(mat), float("nan") if logE is None else float(logE), _dptr(F))
    return F


def cell_keys(cfg: OraConfig, x_soa: np.ndarray):
    """Keys of FP32 positions given as a (3, N) array (one plane per axis)."""
    x_soa = np.ascontiguousarray(x_soa, dtype=np.float32)
    n = x_soa.shape[1]
    keys = np.zeros(n, np.uint32)
    bad = ctypes.c_int32(0)
    lib().ora_cell_keys(ctypes.byref(cfg), n, x_soa.ctypes.data, n, keys.ctypes.data, ctypes.byref(bad))
    return keys, bad.value


def stable_sort(keys: np.ndarray) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    perm = np.zeros(keys.shape[0], np.uint32)
    lib().ora_stable_sort(keys.shape[0], keys.ctypes.data, perm.ctypes.data)
    return perm


class State:
    """FP64 particle state (array of structures)."""

    def __init__(self, x, v, B, F, mat=None, logE=None):
        self.x = np.array(x, dtype=np.float64, order="C").reshape(-1, 3)
        self.v = np.array(v, dtype=np.float64, order="C").reshape(-1, 3)
        self.B = np.array(B, dtype=np.float64, order="C").reshape(-1, 3, 3)
        self.F = np.array(F, dtype=np.float64, order="C").reshape(-1, 3, 3)
        self.mat = None if mat is None else np.ascontiguousarray(mat, dtype=np.uint8)
        self.logE = None if logE is None else np.ascontiguousarray(logE, dtype=np.float64)

    @classmethod
    def from_scene(cls, sc):
        return cls(sc.x, sc.v, sc.B, sc.F, sc.mat, sc.logE)

    def copy(self):
        return State(self.x, self.v, self.B, self.F, self.mat, self.logE)

    @property
    def n(self):
        return self.x.shape[0]


def step(cfg: OraConfig, mats, st: State, dt: float, grids: bool = False):
    """Advance `st` in place by one step.  Returns (status, diag[32], grids-or-None);
    grids = dict(m=[2, ny+1, ... ], p=..., v=...) indexed [g][iz][iy][ix](,3)."""
    n = st.n
    dims = (cfg.n_cells[2] + 1, cfg.n_cells[1] + 1, cfg.n_cells[0] + 1)
    out = OraOutputs()
    diag = np.zeros(32)
    out.diag = diag.ctypes.data
    g = None
    if grids:
        g = dict(m=np.zeros((2,) + dims), p=np.zeros((2,) + dims + (3,)), v=np.zeros((2,) + dims + (3,)))
        out.grid_m, out.grid_p, out.grid_v = g["m"].ctypes.data, g["p"].ctypes.data, g["v"].ctypes.data
    mat_ptr = None if st.mat is None else st.mat.ctypes.data
    loge_ptr = None if st.logE is None else st.logE.ctypes.data
    status = lib().ora_step(ctypes.byref(cfg), mats, len(mats), n, _dptr(st.x), _dptr(st.v), _dptr(st.B),
                            _dptr(st.F), mat_ptr, loge_ptr, float(dt), ctypes.byref(out))
    return status, diag, g


def step_quadratic(cfg: OraConfig, mats, st: State, dt: float, grids: bool = False):
    """One step of the single-grid quadratic B-spline comparison kernel, in place.
    Returns (status, diag[32], grids-or-None) with grids = dict(m, p, v) of the one
    grid, indexed [iz][iy][ix](,3)."""
    n = st.n
    dims = (cfg.n_cells[2] + 1, cfg.n_cells[1] + 1, cfg.n_cells[0] + 1)
    out = OraOutputs()
    diag = np.zeros(32)
    out.diag = diag.ctypes.data
    g = None
    if grids:
        g = dict(m=np.zeros(dims), p=np.zeros(dims + (3,)), v=np.zeros(dims + (3,)))
        out.grid_m, out.grid_p, out.grid_v = g["m"].ctypes.data, g["p"].ctypes.data, g["v"].ctypes.data
    mat_ptr = None if st.mat is None else st.mat.ctypes.data
    loge_ptr = None if st.logE is None else st.logE.ctypes.data
    status = lib().ora_step_quadratic(ctypes.byref(cfg), mats, len(mats), n, _dptr(st.x), _dptr(st.v), _dptr(st.B),
                                      _dptr(st.F), mat_ptr, loge_ptr, float(dt), ctypes.byref(out))
    return status, diag, g


def Nq(r: float) -> float:
    return lib().ora_Nq(float(r))


def num_threads() -> int:
    return lib().ora_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of the checker's parallel loops (for timing; its results are
    the same for any thread count)."""
    lib().ora_set_num_threads(int(n))


def step_vjp(cfg: OraConfig, mats, st: State, dt: float, xb, vb, Bb, Fb):
    """Cotangents of the state entering one step from those of the state it
    produces (fixed corotated, MLS).  Returns (status, dict(x, v, B, F, logE));
    logE is None when the state has no per-particle log modulus."""
    n = st.n
    c = [np.array(a, dtype=np.float64, order="C") for a in (xb, vb, Bb, Fb)]
    out = dict(x=np.zeros((n, 3)), v=np.zeros((n, 3)), B=np.zeros((n, 3, 3)), F=np.zeros((n, 3, 3)))
    out["logE"] = None if st.logE is None else np.zeros(n)
    mat_ptr = None if st.mat is None else st.mat.ctypes.data
    loge_ptr = None if st.logE is None else st.logE.ctypes.data
    status = lib().ora_step_vjp(ctypes.byref(cfg), mats, len(mats), n, _dptr(st.x), _dptr(st.v), _dptr(st.B),
                                _dptr(st.F), mat_ptr, loge_ptr, float(dt), _dptr(c[0]), _dptr(c[1]), _dptr(c[2]),
                                _dptr(c[3]), _dptr(out["x"]), _dptr(out["v"]), _dptr(out["B"]), _dptr(out["F"]),
                                None if out["logE"] is None else out["logE"].ctypes.data)
    return status, out


def particle_masses(mats, st: State) -> np.ndarray:
    idx = np.zeros(st.n, np.int64) if st.mat is None else st.mat.astype(np.int64)
    return np.array([mats[i].rho * mats[i].vol0 for i in range(len(mats))])[idx]


def com_loss(target):
    """Squared distance of the mass-weighted centre of mass to `target`, as a loss
    callable (mats, state) -> (value, dL/dx)."""
    t = np.asarray(target, np.float64)

    def f(mats, st):
        m = particle_masses(mats, st)
        com = (m[:, None] * st.x).sum(axis=0) / m.sum()
        d = com - t
        return float(d @ d), (2.0 * d)[None, :] * (m / m.sum())[:, None]
    return f


def spread_loss(mats, st):
    """Mass-weighted mean squared distance of the particles from their centre of
    mass (depends on how the body deforms, so on its stiffness)."""
    m = particle_masses(mats, st)
    M = m.sum()
    com = (m[:, None] * st.x).sum(axis=0) / M
    r = st.x - com
    return float((m * (r * r).sum(axis=1)).sum() / M), 2.0 * (m / M)[:, None] * r


def rollout_loss(cfg: OraConfig, mats, st0: State, dt: float, nsteps: int, loss) -> float:
    st = st0.copy()
    for _ in range(nsteps):
        status, _, _ = step(cfg, mats, st, dt)
        if status != 0:
            raise RuntimeError("oracle step failed with status %d" % status)
    return loss(mats, st)[0]


def rollout_loss_grad(cfg: OraConfig, mats, st0: State, dt: float, nsteps: int, loss):
    """Loss of an n-step rollout and its gradient with respect to the initial state
    (x, v, B, F) and the per-particle log modulus, by running the steps forward,
    keeping every entering state, and applying step_vjp in reverse."""
    states = [st0.copy()]
    for _ in range(nsteps):
        st = states[-1].copy()
        status, _, _ = step(cfg, mats, st, dt)
        if status != 0:
            raise RuntimeError("oracle step failed with status %d" % status)
        states.append(st)
    value, xb = loss(mats, states[-1])
    n = st0.n
    vb, Bb, Fb = np.zeros((n, 3)), np.zeros((n, 3, 3)), np.zeros((n, 3, 3))
    logEb = None if st0.logE is None else np.zeros(n)
    for k in range(nsteps - 1, -1, -1):
        status, g = step_vjp(cfg, mats, states[k], dt, xb, vb, Bb, Fb)
        if status != 0:
            raise RuntimeError("oracle step_vjp failed with status %d" % status)
        xb, vb, Bb, Fb = g["x"], g["v"], g["B"], g["F"]
        if logEb is not None:
            logEb += g["logE"]
    return value, dict(x=xb, v=vb, B=Bb, F=Fb, logE=logEb)
