"""One-particle transition densities of the DMRG-TDA roots (oracle; test
infrastructure only).

Definition followed (Sec. VI A, with the TDA of Sec. II C-D): for the TDA
eigenvectors Psi^nu of H in the tangent space of the MPS with the reference
removed (orthonormal basis B, H restricted there, unit-norm eigenvectors),
    gamma^nu_pq = <Psi^nu | E_pq | Psi0>,  E_pq = sum_sigma a+_{p sigma} a_{q sigma}.
The sign of each eigenvector is arbitrary.
"""
from __future__ import annotations

import numpy as np

from . import response


def tda_transition(mps, dets, H, Na, Nb, nroots, tol=1e-10):
    """(E0, E_nu for the nroots lowest roots, gamma[nu, p, q])."""
    psi0, B = response.tangent_space(mps, dets, tol)
    e0 = float(psi0 @ (H @ psi0))
    w, U = np.linalg.eigh(B.T @ (H @ B))
    L = mps.L
    gam = np.zeros((nroots, L, L))
    for p in range(L):
        for q in range(L):
            e = np.zeros((L, L))
            e[p, q] = 1.0
            v = B.T @ (response.onebody(e, Na, Nb) @ psi0)
            gam[:, p, q] = U[:, :nroots].T @ v
    return e0, w[:nroots], gam
