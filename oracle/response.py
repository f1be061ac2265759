"""Frequency-dependent linear response of an MPS reference in its tangent
space (oracle; test infrastructure only).

Definition followed (Sec. II B, eqs. realresp and imagresp, with the
first-order wavefunction of eq. psi1st): for a perturbation V the +omega and
-omega components of the first-order wavefunction solve

    (H - (E0 - omega)) Psi1_+ = -Q V Psi0,   (H - (E0 + omega)) Psi1_- = -Q V Psi0,

where Psi1 ranges over the first-order changes of the MPS.  The gauge
conditions of eqs. left-orthoSeb and right-orthoSeb, together with
Psi1 orthogonal to Psi0, make those changes span exactly the tangent space
with the reference removed, so in an orthonormal basis B of that space the
equations read B^T (H - z) B x = -B^T V Psi0 with z = E0 -+ omega, and
chi_pm = <V Psi0 | Psi1_pm> = (B^T V Psi0) . x_pm.  E0 = <Psi0|H|Psi0>.
"""
from __future__ import annotations

import numpy as np

from . import fci, mpsvec, tda


def onebody(v, Na, Nb):
    """Determinant-basis matrix of V = sum_pq v_pq E_pq (spin-summed
    excitation operators): the FCI Hamiltonian with no two-body part."""
    L = v.shape[0]
    _, V = fci.hamiltonian(v, np.zeros((L, L, L, L)), 0.0, Na, Nb)
    return V.toarray()


def tangent_space(mps, dets, tol=1e-10):
    """(Psi0 normalized, orthonormal basis of the tangent space with Psi0
    removed), as in the TDA oracle."""
    psi0 = mpsvec.mps_to_fci(mps, dets)
    psi0 = psi0 / np.linalg.norm(psi0)
    Q, _ = tda.tangent_basis(mps, dets, tol)
    Q = Q - np.outer(psi0, psi0 @ Q)
    U, s, _ = np.linalg.svd(Q, full_matrices=False)
    return psi0, U[:, s > 1e-8]


def response(mps, dets, H, V, omega, tol=1e-10):
    """(chi_+, chi_-) at frequency omega: the two shifted linear systems
    solved in the explicit tangent basis."""
    psi0, B = tangent_space(mps, dets, tol)
    e0 = float(psi0 @ (H @ psi0))
    b = B.T @ (V @ psi0)
    Hs = B.T @ (H @ B)
    eye = np.eye(Hs.shape[0])
    xp = np.linalg.solve(Hs - (e0 - omega) * eye, -b)
    xm = np.linalg.solve(Hs - (e0 + omega) * eye, -b)
    return float(b @ xp), float(b @ xm)
