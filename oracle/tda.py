"""DMRG-TDA by plain Rayleigh-Ritz in the MPS tangent space (oracle; test only).

Definition followed (Sec. II C-D): the TDA is the variational problem
H X = omega S X in the space spanned by the first derivatives of the
reference MPS with respect to its site tensors, with the reference itself
projected out.  In any gauge with full-rank tensors the derivatives with
respect to site i span the columns of the one-site product basis P_i, so the
tangent space is the sum of the column spaces of all P_i.  Its orthogonal
projector comes from the eigenvectors of sum_i P_i P_i^T with non-negligible
eigenvalue (rank threshold), the reference direction is removed, and H is
diagonalized there.  The returned values are total energies E_mu; the
excitation energies are E_mu - E_0 with E_0 = <Psi0|H|Psi0>.
"""
from __future__ import annotations

import numpy as np

from . import mpsvec


def tangent_basis(mps, dets, tol=1e-10):
    """Orthonormal basis of span{dPsi/dA_i} (FCI-space columns) and its rank."""
    n = len(dets)
    G = np.zeros((n, n))
    for i in range(mps.L):
        P = mpsvec.site_basis(mps, dets, i)
        G += P @ P.T
    w, V = np.linalg.eigh(G)
    keep = w > tol * max(w.max(), 1.0)
    return V[:, keep], int(keep.sum())


def redundancy_free_rank(mps):
    """Dimension of the tangent space of an injective MPS: all site-tensor
    parameters minus the gauge freedom of every internal bond (one invertible
    matrix per bond sector)."""
    npar = sum(mps.site_size(i) for i in range(mps.L))
    gauge = sum(d * d for b in range(1, mps.L) for _, d in mps.bonds[b])
    return npar - gauge


def tda_roots(mps, dets, H, nroots, tol=1e-10):
    """Lowest nroots Rayleigh-Ritz energies of H in the tangent space with the
    reference removed; returns (E0, E_mu array)."""
    psi0 = mpsvec.mps_to_fci(mps, dets)
    psi0 = psi0 / np.linalg.norm(psi0)
    Q, _ = tangent_basis(mps, dets, tol)
    Q = Q - np.outer(psi0, psi0 @ Q)
    # re-orthonormalize after removing the reference (one direction drops)
    U, s, _ = np.linalg.svd(Q, full_matrices=False)
    B = U[:, s > 1e-8]
    Hs = B.T @ (H @ B)
    w = np.linalg.eigvalsh(Hs)
    e0 = float(psi0 @ (H @ psi0))
    return e0, w[:nroots]
