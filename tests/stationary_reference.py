"""Stationary MPS references for the RPA tests (test infrastructure).

DMRG-RPA linearizes the time-dependent variational principle around a
stationary point of the energy on the MPS manifold (Sec. II C).  The
two-site sweeps of the library truncate at every bond, so their final MPS
is close to, not at, such a point.  Here a plain one-site DMRG on the CPU
(dense effective Hamiltonians P_i^T H P_i from the oracle, lowest
eigenvector as the new centre tensor, mixed-canonical form rebuilt after
every step) converges a random MPS of fixed bond dimensions until the
energy no longer changes; its gradient on the manifold (the tangent-space
component of (H - E0) Psi0) is then ~1e-7 for the small systems used.
"""
import numpy as np

import synth
from oracle import firstorder, mpsvec, tda


def onesite_ground(mps, dets, H, max_sweeps=200, tol=1e-14):
    """(stationary MPS, energy, sweeps) from one-site sweeps starting at mps."""
    L = mps.L
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    e_old = None
    e = None
    for sweep in range(max_sweeps):
        for i in list(range(L)) + list(range(L - 2, 0, -1)):
            P = mpsvec.site_basis(mps, dets, i)
            He = P.T @ (Hd @ P)
            w, V = np.linalg.eigh(0.5 * (He + He.T))
            c = firstorder.blocks(mps, i, V[:, 0])
            A = [mps.Lt[j] if j < i else (c if j == i else mps.Rt[j]) for j in range(L)]
            mps = synth.canonical_from_tensors(L, mps.Na, mps.Nb, mps.bonds, A)
            e = float(w[0])
        if e_old is not None and abs(e - e_old) < tol:
            break
        e_old = e
    return mps, e, sweep + 1


def gradient_norm(mps, dets, H):
    """|P_T (H - E0) Psi0|: the gradient of the energy on the manifold."""
    psi = mpsvec.mps_to_fci(mps, dets)
    psi /= np.linalg.norm(psi)
    e0 = float(psi @ (H @ psi))
    T, _ = tda.tangent_basis(mps, dets)
    return float(np.linalg.norm(T.T @ (H @ psi - e0 * psi)))
