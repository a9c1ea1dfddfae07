"""Oracle gradient of a PCG-solved loss w.r.t. per-cell log-coefficients (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The operator is the cell-centred finite-volume diffusion matrix with
harmonic-mean face coefficients a_f = 2 kL kR / (kL + kR) and zero-Dirichlet
ghost faces of coefficient 2 kc, kappa = exp(theta).  Boundary conditions:
``bc="dirichlet"`` puts such a ghost face on every boundary face;
``bc="x0"`` (problem A of Section 7: one Dirichlet face, the rest Neumann)
keeps only the ghost faces on the x = 0 face (x is the last, fastest
array axis) and leaves every other boundary face without flux.  Its assembly is written
here independently of the input generators so that the derivative below is
checked against this module's own operator.

For L(u), u = A(kappa)^{-1} f, the adjoint identity gives
dL/dtheta_c = -kappa_c * lambda^T (dA/dkappa_c) u with A lambda = dL/du.
Differentiating the face terms a_f (e_L - e_R)(e_L - e_R)^T and
b_f e_c e_c^T:
  d a_f / d kL = 2 kR^2 / (kL + kR)^2,   d b_f / d kc = 2,
so per cell c
  g_c = -kappa_c [ sum_{faces f=(L,R) containing c} (d a_f/d kappa_c)(lam_L - lam_R)(u_L - u_R)
                   + sum_{boundary faces of c} 2 lam_c u_c ].
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


BCS = ("dirichlet", "x0")


def _ghost_ends(ndim: int, ax: int, bc: str):
    """Which ends (low, high) of axis ``ax`` carry a Dirichlet ghost face."""
    if bc not in BCS:
        raise ValueError(f"bc must be one of {BCS}")
    if bc == "dirichlet":
        return True, True
    return ax == ndim - 1, False


def assemble_cc(kappa: np.ndarray, bc: str = "dirichlet") -> sp.csr_matrix:
    """Harmonic-mean cell-centred operator (oracle's own assembly)."""
    kappa = np.asarray(kappa, dtype=np.float64)
    shape = kappa.shape
    n = kappa.size
    idx = np.arange(n).reshape(shape)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for ax in range(kappa.ndim):
        L = np.moveaxis(kappa, ax, 0)
        I = np.moveaxis(idx, ax, 0)
        kl, kr = L[:-1], L[1:]
        a = (2.0 * kl * kr / (kl + kr)).ravel()
        il, ir = I[:-1].ravel(), I[1:].ravel()
        np.add.at(diag, il, a)
        np.add.at(diag, ir, a)
        rows += [il, ir]
        cols += [ir, il]
        vals += [-a, -a]
        lo, hi = _ghost_ends(kappa.ndim, ax, bc)
        if lo:
            np.add.at(diag, I[0].ravel(), 2.0 * L[0].ravel())
        if hi:
            np.add.at(diag, I[-1].ravel(), 2.0 * L[-1].ravel())
    rows.append(np.arange(n)); cols.append(np.arange(n)); vals.append(diag)
    M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    M.sort_indices()
    return M


def coeff_grad_cc(kappa: np.ndarray, u: np.ndarray, lam: np.ndarray, bc: str = "dirichlet") -> np.ndarray:
    """Per-cell -kappa_c * lam^T (dA/dkappa_c) u, returned in grid shape."""
    kappa = np.asarray(kappa, dtype=np.float64)
    U = np.asarray(u, dtype=np.float64).reshape(kappa.shape)
    Lm = np.asarray(lam, dtype=np.float64).reshape(kappa.shape)
    acc = np.zeros(kappa.shape)
    for ax in range(kappa.ndim):
        K = np.moveaxis(kappa, ax, 0)
        Uu = np.moveaxis(U, ax, 0)
        Ll = np.moveaxis(Lm, ax, 0)
        G = np.moveaxis(acc, ax, 0)  # view into acc
        kl, kr = K[:-1], K[1:]
        s2 = (kl + kr) ** 2
        jump = (Ll[:-1] - Ll[1:]) * (Uu[:-1] - Uu[1:])
        G[:-1] += 2.0 * kr ** 2 / s2 * jump
        G[1:] += 2.0 * kl ** 2 / s2 * jump
        lo, hi = _ghost_ends(kappa.ndim, ax, bc)
        if lo:
            G[0] += 2.0 * Ll[0] * Uu[0]
        if hi:
            G[-1] += 2.0 * Ll[-1] * Uu[-1]
    return -kappa * acc
