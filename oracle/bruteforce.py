"""Definition-level brute-force step for tiny scenes (TEST INFRASTRUCTURE ONLY).

A second, independent transcription of the paper's step used to pin the C++
oracle: it evaluates the tensor-product compact kernel of section 4.2 against
*every* node of both staggered grids (no stencil, no cell lookup), keeps the
grids as dense numpy arrays, and takes singular value decompositions from
LAPACK (numpy.linalg.svd).  Cost is O(particles x nodes), so it is only used
with a few hundred particles on grids of about 8^3 cells.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def K1(r):
    """Section 4.1: 1 - |r| + sin(2 pi |r|)/(2 pi) inside |r| < 1, zero outside."""
    a = np.abs(r)
    return np.where(a < 1.0, 1.0 - a + np.sin(TWO_PI * a) / TWO_PI, 0.0)


def dK1(r):
    a = np.abs(r)
    return np.where(a < 1.0, np.sign(r) * (np.cos(TWO_PI * a) - 1.0), 0.0)


def node_positions(n_cells, dx, origin, k):
    """All nodes of grid G_k: world position origin + (i + k/4) dx, i in [0, n]^3,
    flattened with x fastest."""
    axes = [origin[a] + (np.arange(n_cells[a] + 1) + k / 4.0) * dx for a in range(3)]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def rv_svd(F):
    """Rotation-variant SVD from LAPACK: det U = det V = +1, sign on the last value."""
    U, S, Vh = np.linalg.svd(F)
    S = S.copy()
    if np.linalg.det(U) < 0:
        U = U.copy()
        U[:, 2] *= -1
        S[2] *= -1
    if np.linalg.det(Vh) < 0:
        Vh = Vh.copy()
        Vh[2, :] *= -1
        S[2] *= -1
    return U, S, Vh.T


def lame(E, nu):
    return E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))


def tau_of(model, E, nu, F):
    mu, lam = lame(E, nu)
    U, S, V = rv_svd(F)
    if model == 0:
        R = U @ V.T
        J = np.linalg.det(F)
        return 2 * mu * (F - R) @ F.T + lam * (J - 1) * J * np.eye(3)
    eps = np.log(np.maximum(S, 1e-4))
    return U @ np.diag(2 * mu * eps + lam * eps.sum()) @ U.T


def dp_project(E, nu, phi_deg, F):
    mu, lam = lame(E, nu)
    U, S, V = rv_svd(F)
    sphi = math.sin(math.radians(phi_deg))
    alpha = math.sqrt(2.0 / 3.0) * 2 * sphi / (3 - sphi)
    eps = np.log(np.maximum(S, 1e-4))
    tr = eps.sum()
    dev = eps - tr / 3
    dn = np.linalg.norm(dev)
    if tr > 0 or dn == 0:
        Sn = np.ones(3)
    else:
        dg = dn + (3 * lam + 2 * mu) / (2 * mu) * tr * alpha
        if dg <= 0:
            return F.copy()
        Sn = np.exp(eps - dg * dev / dn)
    return U @ np.diag(Sn) @ V.T


def step(sc, x, v, B, F, dt, mats=None, transfer="mls"):
    """One step on all nodes of both grids, transfer "mls" (section 4.5), "apic"
    (section 4.4, exact kernel gradients) or "pic" (section 4.3: no affine term,
    exact gradients, B not carried).  Inputs are FP64 arrays (N,3), (N,3,3);
    returns dict(x, v, B, F, m[2,nodes], p[2,nodes,3], vt[2,nodes,3])."""
    mats = sc.materials if mats is None else mats
    n_cells, dx, origin = sc.n_cells, sc.dx, np.asarray(sc.origin, np.float64)
    N = x.shape[0]
    mat = sc.mat if sc.mat is not None else np.zeros(N, np.uint8)
    mp = np.array([mats[m].rho * mats[m].vol0 for m in mat])
    V0 = np.array([mats[m].vol0 for m in mat])
    grids = []
    for k in (-1.0, 1.0):
        xi = node_positions(n_cells, dx, origin, k)              # (Nn, 3)
        d = xi[None, :, :] - x[:, None, :]                       # (N, Nn, 3)
        r = d / dx
        wa = K1(r)
        w = wa[..., 0] * wa[..., 1] * wa[..., 2]                 # (N, Nn)
        dwa = -dK1(r) / dx
        gw = np.stack([dwa[..., 0] * wa[..., 1] * wa[..., 2], wa[..., 0] * dwa[..., 1] * wa[..., 2],
                       wa[..., 0] * wa[..., 1] * dwa[..., 2]], axis=-1)
        grids.append((k, xi, d, w, gw))
    D = sum(0.5 * np.einsum("pn,pna,pnb->pab", w, d, d) for (_, _, d, w, _) in grids)
    Dinv = np.linalg.inv(D)
    tau = np.stack([tau_of(mats[mat[p]].model, mats[mat[p]].E, mats[mat[p]].nu, F[p]) for p in range(N)])
    out = dict(m=[], p=[], vt=[])
    vts = []
    for (k, xi, d, w, gw) in grids:
        m = w.T @ mp
        BD = np.zeros_like(B) if transfer == "pic" else np.einsum("pab,pbc->pac", B, Dinv)
        mom = np.einsum("pn,p,pna->na", w, mp, v[:, None, :] + np.einsum("pab,pnb->pna", BD, d))
        if transfer == "mls":
            grad = np.einsum("pn,pab,pnb->pna", w, Dinv, d)
        else:
            grad = gw
        f = -np.einsum("p,pab,pnb->na", V0, tau, grad)
        p = mom + dt * f
        vt = np.zeros_like(p)
        pos = m > 0
        vt[pos] = p[pos] / m[pos, None] + dt * np.asarray(sc.gravity)[None, :]
        if sc.bc_band > 0:
            cells = (xi - origin[None, :]) / dx
            stick = np.any((cells < sc.bc_band) | (cells > np.asarray(n_cells)[None, :] - sc.bc_band), axis=1)
            vt[stick] = 0.0
        out["m"].append(m)
        out["p"].append(p)
        out["vt"].append(vt)
        vts.append(vt)
    vnew = sum(0.5 * np.einsum("pn,na->pa", w, vt) for (_, _, _, w, _), vt in zip(grids, vts))
    Bnew = sum(0.5 * np.einsum("pn,na,pnb->pab", w, vt, d) for (_, _, d, w, _), vt in zip(grids, vts))
    if transfer == "mls":
        C = np.einsum("pab,pbc->pac", Bnew, Dinv)
    else:
        C = sum(0.5 * np.einsum("na,pnb->pab", vt, gw) for (_, _, _, _, gw), vt in zip(grids, vts))
    Fn = np.einsum("pab,pbc->pac", np.eye(3)[None] + dt * C, F)
    for p in range(N):
        mt = mats[mat[p]]
        if mt.model == 1:
            Fn[p] = dp_project(mt.E, mt.nu, mt.friction_deg, Fn[p])
    if transfer == "pic":
        Bnew = np.zeros_like(Bnew)
    return dict(x=x + dt * vnew, v=vnew, B=Bnew, F=Fn, m=np.stack(out["m"]), p=np.stack(out["p"]),
                vt=np.stack(out["vt"]))


def Nq(r):
    """Quadratic B-spline: 3/4 - r^2 (|r| < 1/2), (3/2 - |r|)^2 / 2 (1/2 <= |r| < 3/2)."""
    a = np.abs(r)
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def step_quadratic(sc, x, v, B, F, dt, mats=None):
    """One step of the single-grid quadratic B-spline comparison kernel against every
    node of the grid (node i at origin + i dx).  Same return layout as `step`, with
    m, p, vt of the one grid."""
    mats = sc.materials if mats is None else mats
    n_cells, dx, origin = sc.n_cells, sc.dx, np.asarray(sc.origin, np.float64)
    N = x.shape[0]
    mat = sc.mat if sc.mat is not None else np.zeros(N, np.uint8)
    mp = np.array([mats[m].rho * mats[m].vol0 for m in mat])
    V0 = np.array([mats[m].vol0 for m in mat])
    xi = node_positions(n_cells, dx, origin, 0.0)
    d = xi[None, :, :] - x[:, None, :]
    wa = Nq(d / dx)
    w = wa[..., 0] * wa[..., 1] * wa[..., 2]
    D = np.einsum("pn,pna,pnb->pab", w, d, d)
    Dinv = np.linalg.inv(D)
    tau = np.stack([tau_of(mats[mat[p]].model, mats[mat[p]].E, mats[mat[p]].nu, F[p]) for p in range(N)])
    m = w.T @ mp
    Q = np.einsum("pab,pbc->pac", mp[:, None, None] * B - dt * V0[:, None, None] * tau, Dinv)
    p = np.einsum("pn,pna->na", w, mp[:, None, None] * v[:, None, :] + np.einsum("pab,pnb->pna", Q, d))
    vt = np.zeros_like(p)
    pos = m > 0
    vt[pos] = p[pos] / m[pos, None] + dt * np.asarray(sc.gravity)[None, :]
    if sc.bc_band > 0:
        cells = (xi - origin[None, :]) / dx
        stick = np.any((cells < sc.bc_band) | (cells > np.asarray(n_cells)[None, :] - sc.bc_band), axis=1)
        vt[stick] = 0.0
    vnew = np.einsum("pn,na->pa", w, vt)
    Bnew = np.einsum("pn,na,pnb->pab", w, vt, d)
    C = np.einsum("pab,pbc->pac", Bnew, Dinv)
    Fn = np.einsum("pab,pbc->pac", np.eye(3)[None] + dt * C, F)
    for q in range(N):
        mt = mats[mat[q]]
        if mt.model == 1:
            Fn[q] = dp_project(mt.E, mt.nu, mt.friction_deg, Fn[q])
    return dict(x=x + dt * vnew, v=vnew, B=Bnew, F=Fn, m=m, p=p, vt=vt)
