"""Host-side diagnostics of simulation results (analysis of read-back state, not part
of the step): kinetic and elastic energy of a fixed-corotated body, for the
numerical-diffusion comparison of kernels."""
from __future__ import annotations

import numpy as np


def energies(v, F, mass, vol0, E, nu):
    """(kinetic, elastic) energy of particles with velocities v (N, 3), deformation
    gradients F (N, 3, 3), particle mass and reference volume, and fixed-corotated
    modulus E, ratio nu: kinetic 1/2 sum m |v|^2, elastic sum V0 psi(F) with
    psi = mu |F - R|^2 + lambda/2 (J - 1)^2 and R the rotation of the polar
    decomposition (rotation-variant SVD: det R = +1)."""
    v = np.asarray(v, np.float64)
    F = np.asarray(F, np.float64)
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    U, S, Vh = np.linalg.svd(F)
    flip = np.linalg.det(U) * np.linalg.det(Vh) < 0
    U[flip, :, 2] *= -1.0
    R = U @ Vh
    J = np.linalg.det(F)
    psi = mu * ((F - R) ** 2).sum(axis=(1, 2)) + 0.5 * lam * (J - 1.0) ** 2
    return 0.5 * mass * float((v * v).sum()), vol0 * float(psi.sum())
