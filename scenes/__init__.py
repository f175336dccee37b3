"""Seeded synthetic scenes for the compact-kernel MPM step.

This module only *generates inputs*: particle positions, velocities, affine
matrices, deformation gradients and material tags, plus the plain scene
parameters (grid size, spacing, time step, material constants).  It holds none
of the method's arithmetic (no kernel weights, no transfers, no stress), so the
FP64 oracle and the HIP path can both consume its output without sharing any
computation.

Sampling follows the paper's workloads: solids seeded at 8 particles per cell
(section 6.1 uses 8 ppc; section 6.2 samples solids uniformly in 256^3-class
grids).  The paper's meshes are not available, so every scene is a box (or a
sphere) filled by stratified jitter: each dx^3 region is split into 2x2x2
sub-cells and one particle is drawn uniformly inside each sub-cell, with numpy's
PCG64 generator and a fixed seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

FIXED_COROTATED = 0
DRUCKER_PRAGER = 1


@dataclasses.dataclass
class Material:
    model: int
    E: float
    nu: float
    rho: float
    vol0: float
    friction_deg: float = 30.0


@dataclasses.dataclass
class Scene:
    name: str
    n_cells: tuple
    dx: float
    origin: tuple
    gravity: tuple
    bc_band: int
    dt: float
    steps: int
    materials: List[Material]
    x: np.ndarray            # (N, 3) float32, world positions
    v: np.ndarray            # (N, 3) float32
    B: np.ndarray            # (N, 3, 3) float32, APIC affine matrix
    F: np.ndarray            # (N, 3, 3) float32, deformation gradient
    mat: np.ndarray          # (N,) uint8 material index
    logE: Optional[np.ndarray] = None   # (N,) float32, optional per-particle log Young's modulus

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def copy(self) -> "Scene":
        return dataclasses.replace(
            self, x=self.x.copy(), v=self.v.copy(), B=self.B.copy(), F=self.F.copy(),
            mat=self.mat.copy(), logE=None if self.logE is None else self.logE.copy())


def stratified_box(rng: np.random.Generator, lo, ncell, dx) -> np.ndarray:
    """Positions filling an axis-aligned box of ncell = (cx, cy, cz) dx-cells whose
    lower corner is `lo`: 2x2x2 sub-cells per cell, one uniform sample in each.
    Particle order is x fastest, then y, then z (sub-cells inside each cell)."""
    cx, cy, cz = (int(c) for c in ncell)
    iz, iy, ix = np.meshgrid(np.arange(cz), np.arange(cy), np.arange(cx), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    sub = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=np.float64)
    pts = (cells[:, None, :] + (sub[None, :, :] + rng.random((cells.shape[0], 8, 3))) * 0.5)
    want = np.floor(pts.reshape(-1, 3))
    lo = np.asarray(lo, dtype=np.float64)
    out = (pts.reshape(-1, 3) * dx + lo).astype(np.float32)
    # rounding to FP32 may push a sample onto its cell's upper face: step it back inside
    over = np.floor((out.astype(np.float64) - lo) / dx) > want
    out[over] = np.nextafter(out[over], np.float32(-np.inf))
    return out


def _rest_state(n: int):
    v = np.zeros((n, 3), np.float32)
    B = np.zeros((n, 3, 3), np.float32)
    F = np.tile(np.eye(3, dtype=np.float32), (n, 1, 1))
    return v, B, F


def cube_elastic(seed: int = 0) -> Scene:
    """A 16^3-cell elastic cube (32,768 particles) centred at (0.5, 0.6, 0.5) on a
    32^3 grid over the unit box, falling at 1 m/s: fixed-corotated, rho=1000,
    E=1e4, nu=0.3, gravity -9.8, sticky walls, dt=1e-4, 100 steps."""
    dx = 1.0 / 32
    rng = np.random.Generator(np.random.PCG64(seed))
    x = stratified_box(rng, (0.25, 0.35, 0.25), (16, 16, 16), dx)
    v, B, F = _rest_state(x.shape[0])
    v[:, 1] = -1.0
    mats = [Material(FIXED_COROTATED, 1e4, 0.3, 1000.0, dx ** 3 / 8)]
    return Scene("cube_elastic_32k", (32, 32, 32), dx, (0.0, 0.0, 0.0), (0.0, -9.8, 0.0), 2,
                 1e-4, 100, mats, x, v, B, F, np.zeros(x.shape[0], np.uint8))


def cube_elastic_perturbed(seed: int = 1, floor_cells: Optional[float] = None) -> Scene:
    """The elastic cube with seeded perturbations so that stress, the affine
    term and plasticity-free rotation all take part: v += 0.1 N(0,1),
    F = I + 0.01 N(0,1).  With `floor_cells` the cube's bottom face is placed at
    that height (in cells) so its lowest particles reach the sticky wall band."""
    sc = cube_elastic(0)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = sc.n
    sc.v = (sc.v + 0.1 * rng.standard_normal((n, 3))).astype(np.float32)
    sc.F = (np.eye(3)[None] + 0.01 * rng.standard_normal((n, 3, 3))).astype(np.float32)
    sc.name = "cube_elastic_perturbed"
    if floor_cells is not None:
        shift = floor_cells * sc.dx - 0.35
        sc.x = (sc.x.astype(np.float64) + np.array([0.0, shift, 0.0])).astype(np.float32)
        sc.name = "cube_elastic_perturbed_floor"
    return sc


def sand_column(seed: int = 2, scale: int = 1) -> Scene:
    """Drucker-Prager sand column resting on the sticky floor of a 256^3 grid
    (dx = 1/256): cells [96,160) x [2,130) x [96,160), 8 ppc, 4,194,304 particles,
    friction angle 30 deg, E=3.5e5, nu=0.3, rho=1600, dt=2e-5.

    `scale` > 1 shrinks the column footprint by that factor per axis (same grid,
    same material) to give CPU-sized versions of the same workload."""
    n = 256
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    ext = (64 // scale, 128 // scale, 64 // scale)
    lo_cells = (128 - ext[0] // 2, 2, 128 - ext[2] // 2)
    x = stratified_box(rng, tuple(c * dx for c in lo_cells), ext, dx)
    v, B, F = _rest_state(x.shape[0])
    mats = [Material(DRUCKER_PRAGER, 3.5e5, 0.3, 1600.0, dx ** 3 / 8, 30.0)]
    return Scene("sand_column_%d" % x.shape[0], (n, n, n), dx, (0.0, 0.0, 0.0), (0.0, -9.8, 0.0), 2,
                 2e-5, 500, mats, x, v, B, F, np.zeros(x.shape[0], np.uint8))


def diff_box(seed: int = 5, scale: int = 1) -> Scene:
    """The differentiation workload: a 32x16x16-cell elastic box at 8 ppc (65,536
    particles) centred in a 64^3 grid (dx = 1/64), fixed corotated E = 5e4, nu = 0.3,
    rho = 1000, initial velocity N(0, 0.1^2) per component, a per-particle log
    Young's modulus field starting at log 5e4, gravity -9.8, sticky walls, dt = 1e-4,
    64 steps.  `scale` k shrinks the box k-fold per axis and the grid to 64/k cells
    (at least 16) at the same dx, for CPU-sized versions."""
    dx = 1.0 / 64
    n = max(16, 64 // scale)
    ext = (max(1, 32 // scale), max(1, 16 // scale), max(1, 16 // scale))
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = tuple((n / 2 - e / 2) * dx for e in ext)
    x = stratified_box(rng, lo, ext, dx)
    v, B, F = _rest_state(x.shape[0])
    v = (0.1 * rng.standard_normal(v.shape)).astype(np.float32)
    mats = [Material(FIXED_COROTATED, 5e4, 0.3, 1000.0, dx ** 3 / 8)]
    logE = np.full(x.shape[0], np.log(5e4), np.float32)
    return Scene("diff_box_%d" % x.shape[0], (n, n, n), dx, (0.0, 0.0, 0.0), (0.0, -9.8, 0.0), 2,
                 1e-4, 64, mats, x, v, B, F, np.zeros(x.shape[0], np.uint8), logE)


def diff_target(seed: int = 5, scale: int = 1) -> np.ndarray:
    """Target point of the differentiation workload's centre-of-mass loss, uniform in
    the middle 40 % of the domain per axis ([0.3, 0.7]^3 of the unit box)."""
    n = max(16, 64 // scale)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    return (0.3 + 0.4 * rng.random(3)) * (n / 64.0)


def stress_scene(seed: int = 3, sand_cells: int = 3_190_000, scale: int = 1) -> Scene:
    """The stress-scale workload on a 1024^3 virtual grid (dx = 1/1024): seeded random
    axis-aligned sand boxes (sides uniform in [0.03, 0.15], Drucker-Prager as the sand
    column) stacked on the floor by a height map until about `sand_cells` cells are
    covered (~25.5M particles at 8 ppc), and an elastic sphere of radius 0.05
    (fixed corotated, E = 1e7, nu = 0.3, rho = 2000, ~4.5M particles) moving at
    20 m/s along +x towards the stacks; dt = 5e-6, 200 steps.  Boxes are placed in
    x, z in [0.35, 0.9], each resting on the highest column under its footprint, so
    they never overlap.  `scale` k divides every length (and the sand volume) by k
    on a 1024/k grid at the same dx, for smaller versions."""
    n = 1024 // scale
    dx = 1.0 / 1024
    rng = np.random.Generator(np.random.PCG64(seed))
    height = np.full((n, n), 2, np.int64)          # first free cell per (x, z) column, above the wall band
    boxes = []
    covered = 0
    lo_xz, hi_xz = int(0.35 * n), int(0.9 * n)
    while covered < sand_cells // (scale ** 3):
        side = np.maximum(1, np.round(rng.uniform(0.03, 0.15, 3) * 1024 / scale).astype(np.int64))
        x0 = int(rng.integers(lo_xz, max(lo_xz + 1, hi_xz - side[0])))
        z0 = int(rng.integers(lo_xz, max(lo_xz + 1, hi_xz - side[2])))
        y0 = int(height[x0:x0 + side[0], z0:z0 + side[2]].max())
        if y0 + side[1] > n - 8:
            continue
        height[x0:x0 + side[0], z0:z0 + side[2]] = y0 + side[1]
        boxes.append(((x0, y0, z0), tuple(int(c) for c in side)))
        covered += int(side.prod())
    parts = [stratified_box(rng, tuple(c * dx for c in lo), ext, dx) for lo, ext in boxes]
    sand = np.concatenate(parts) if parts else np.zeros((0, 3), np.float32)
    ball = sphere(rng, (0.2 / scale, 0.12 / scale, 0.6 / scale), 0.05 / scale, dx)
    x = np.concatenate([sand, ball]).astype(np.float32)
    v, B, F = _rest_state(x.shape[0])
    v[sand.shape[0]:, 0] = 20.0
    mat = np.zeros(x.shape[0], np.uint8)
    mat[sand.shape[0]:] = 1
    mats = [Material(DRUCKER_PRAGER, 3.5e5, 0.3, 1600.0, dx ** 3 / 8, 30.0),
            Material(FIXED_COROTATED, 1e7, 0.3, 2000.0, dx ** 3 / 8)]
    return Scene("stress_%d" % x.shape[0], (n, n, n), dx, (0.0, 0.0, 0.0), (0.0, -9.8, 0.0), 2,
                 5e-6, 200, mats, x, v, B, F, mat)


def diffusion_cuboid(seed: int = 6, scale: int = 1) -> Scene:
    """Numerical-diffusion scene: a cuboid of 20 x 10 x 140 cells (dx = 1/256) at 8 ppc
    (224,000 particles) centred in a 256^3 grid, at rest except for the velocity
    0.2 sin(500 z) along y (z in metres); fixed corotated, E = 1e5, nu = 0.3,
    rho = 1000 (the material is not stated for this experiment); no gravity;
    dt = 2e-5, 500 steps (100 frames at 10,000 frames per second).  `scale` k
    shortens the cuboid's z extent k-fold."""
    n = 256
    dx = 1.0 / n
    ext = (20, 10, max(4, 140 // scale))
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = tuple((n / 2 - e / 2) * dx for e in ext)
    x = stratified_box(rng, lo, ext, dx)
    v, B, F = _rest_state(x.shape[0])
    v[:, 1] = (0.2 * np.sin(500.0 * x[:, 2].astype(np.float64))).astype(np.float32)
    mats = [Material(FIXED_COROTATED, 1e5, 0.3, 1000.0, dx ** 3 / 8)]
    return Scene("diffusion_cuboid_%d" % x.shape[0], (n, n, n), dx, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 2,
                 2e-5, 500, mats, x, v, B, F, np.zeros(x.shape[0], np.uint8))


def random_blob(seed: int, n_cells=(8, 8, 8), lo_cells=(2.5, 2.5, 2.5), ext_cells=(3, 3, 3),
                model: int = FIXED_COROTATED, v_scale=0.5, B_scale=2.0, F_scale=0.05,
                gravity=(0.0, 0.0, 0.0), bc_band: int = 0, dt: float = 1e-3,
                E: float = 1e4, nu: float = 0.3, rho: float = 1000.0,
                dx: Optional[float] = None, ppc_sub: int = 2) -> Scene:
    """Small random scene for transfer identities and brute-force checks:
    stratified particles in a box of `ext_cells` cells starting at `lo_cells`,
    random v, B and F = I + F_scale N(0,1).  dx defaults to 1/n_cells[0]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dx = (1.0 / n_cells[0]) if dx is None else dx
    x = stratified_box(rng, tuple(c * dx for c in lo_cells), ext_cells, dx)
    n = x.shape[0]
    v = (v_scale * rng.standard_normal((n, 3))).astype(np.float32)
    B = (B_scale * dx * rng.standard_normal((n, 3, 3))).astype(np.float32)
    F = (np.eye(3)[None] + F_scale * rng.standard_normal((n, 3, 3))).astype(np.float32)
    mats = [Material(model, E, nu, rho, dx ** 3 / 8, 30.0)]
    return Scene("random_blob_s%d" % seed, tuple(n_cells), dx, (0.0, 0.0, 0.0), tuple(gravity), bc_band,
                 dt, 1, mats, x, v, B, F, np.zeros(n, np.uint8))


def sphere(rng: np.random.Generator, centre, radius, dx) -> np.ndarray:
    """Stratified samples of a ball: the stratified lattice of its bounding box,
    kept where the sample lies inside the ball."""
    ncell = int(math.ceil(2 * radius / dx)) + 1
    lo = np.asarray(centre, np.float64) - ncell * dx / 2
    pts = stratified_box(rng, lo, (ncell, ncell, ncell), dx).astype(np.float64)
    keep = np.sum((pts - np.asarray(centre)) ** 2, axis=1) < radius * radius
    return pts[keep].astype(np.float32)


@dataclasses.dataclass
class JobSpec:
    """One job of the serving workload: everything needed to build its scene."""
    index: int
    seed: int
    n_target: int        # drawn particle count
    side: int            # box side in cells (the box holds side^3 cells at 8 ppc)
    grid: int            # cells per axis of the job's grid
    sand: bool           # Drucker-Prager sand at rest on the floor, else a falling elastic cube
    nsteps: int
    arrival: float       # seconds after the first arrival (Poisson process of unit rate)


def serving_workload(seed: int = 4, n_jobs: int = 256, nsteps: int = 200,
                     n_min: float = 1e3, n_max: float = 2e6) -> List[JobSpec]:
    """Job mix of the serving benchmark: particle counts log-uniform in
    [n_min, n_max], each a box of N/8 cells at 8 ppc on the smallest power-of-two
    grid in {32, 64, 128, 256} that holds twice the box side plus 8 cells; a fair
    coin picks a falling elastic cube or sand resting on the floor; arrival times
    are a Poisson process of unit rate (scale them to the wanted rate)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    t = 0.0
    for i in range(n_jobs):
        n_target = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        side = max(2, int(round((n_target / 8.0) ** (1.0 / 3.0))))
        grid = next((g for g in (32, 64, 128, 256) if g >= 2 * side + 8), 256)
        sand = bool(rng.random() < 0.5)
        if i > 0:
            t += float(rng.exponential(1.0))
        out.append(JobSpec(i, int(rng.integers(0, 2 ** 31 - 1)), n_target, side, grid, sand, nsteps, t))
    return out


def serving_job(spec: JobSpec) -> Scene:
    """Scene of one serving job.  Elastic: fixed-corotated (rho=1000, E=1e4,
    nu=0.3), centred, falling at 1 m/s, dt=1e-4.  Sand: Drucker-Prager (phi=30 deg,
    rho=1600, E=3.5e5, nu=0.3) on the floor band, at rest, dt=2e-5.  Gravity -9.8,
    sticky walls two cells thick."""
    n = spec.grid
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    s = spec.side
    if spec.sand:
        lo_cells = ((n - s) // 2, 2, (n - s) // 2)
    else:
        lo_cells = ((n - s) // 2, (n - s) // 2, (n - s) // 2)
    x = stratified_box(rng, tuple(c * dx for c in lo_cells), (s, s, s), dx)
    v, B, F = _rest_state(x.shape[0])
    if spec.sand:
        mats = [Material(DRUCKER_PRAGER, 3.5e5, 0.3, 1600.0, dx ** 3 / 8, 30.0)]
        dt = 2e-5
    else:
        v[:, 1] = -1.0
        mats = [Material(FIXED_COROTATED, 1e4, 0.3, 1000.0, dx ** 3 / 8, 30.0)]
        dt = 1e-4
    return Scene("job_%d" % spec.index, (n, n, n), dx, (0.0, 0.0, 0.0), (0.0, -9.8, 0.0), 2, dt, spec.nsteps,
                 mats, x, v, B, F, np.zeros(x.shape[0], np.uint8))


PRESETS = {
    "cube_elastic": cube_elastic,
    "cube_elastic_perturbed": lambda: cube_elastic_perturbed(1),
    "cube_elastic_floor": lambda: cube_elastic_perturbed(1, floor_cells=2.5),
    "sand_column": sand_column,
}
