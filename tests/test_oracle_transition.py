"""Pins of the oracle's TDA transition densities (Sec. VI A): the FCI
transition densities of the excited states when the reference is exact at
full bond dimension (the tangent space is then the whole complement of the
ground state), zero trace (E_pp summed is the particle number, and the roots
are orthogonal to Psi0), and a planted transposition caught."""
import numpy as np

import synth
from oracle import fci, mpsvec, response, transition


def _exact(L, Na, Nb, seed):
    h, eri, e0 = synth.random_integrals(L, seed=seed, K=L, diag_lo=-2, diag_hi=0)
    dets, H, w, vec = fci.fci(h, eri, e0, Na, Nb, nroots=len(fci.determinants(L, Na, Nb)))
    bonds, A = mpsvec.fci_to_mps(vec[:, 0], dets, L, Na, Nb)
    mps = synth.canonical_from_tensors(L, Na, Nb, bonds, A)
    return mps, dets, H, w, vec


def _fci_gamma(vec, L, Na, Nb, n):
    out = np.zeros((n, L, L))
    for p in range(L):
        for q in range(L):
            e = np.zeros((L, L))
            e[p, q] = 1.0
            out[:, p, q] = vec[:, 1:n + 1].T @ (response.onebody(e, Na, Nb) @ vec[:, 0])
    return out


def _align(g, ref):
    # the sign of each root is arbitrary
    s = np.sign(np.sum(g * ref, axis=(1, 2)))
    return g * s[:, None, None]


def test_exact_reference_gives_fci_transition_densities():
    L, Na, Nb = 5, 2, 2
    mps, dets, H, w, vec = _exact(L, Na, Nb, 31)
    e0, ev, g = transition.tda_transition(mps, dets, H, Na, Nb, 4)
    assert abs(e0 - w[0]) < 1e-10
    np.testing.assert_allclose(ev, w[1:5], atol=1e-9)
    assert np.min(np.diff(w[:6])) > 1e-6  # non-degenerate: the vectors are unique up to sign
    ref = _fci_gamma(vec, L, Na, Nb, 4)
    np.testing.assert_allclose(_align(g, ref), ref, atol=1e-9)


def test_transition_density_has_zero_trace_on_truncated_mps():
    L, Na, Nb, M = 6, 3, 3, 12
    h, eri, e0 = synth.random_integrals(L, seed=11, K=6, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, M, seed=12)
    dets, H = fci.hamiltonian(h, eri, e0, Na, Nb)
    _, _, g = transition.tda_transition(mps, dets, H, Na, Nb, 3)
    for nu in range(3):
        assert abs(np.trace(g[nu])) < 1e-10
        assert np.sum(g[nu] ** 2) > 1e-6


def test_planted_transposition_is_caught():
    # gamma_qp in place of gamma_pq differs from the FCI transition density
    L, Na, Nb = 5, 2, 2
    mps, dets, H, w, vec = _exact(L, Na, Nb, 31)
    _, _, g = transition.tda_transition(mps, dets, H, Na, Nb, 2)
    ref = _fci_gamma(vec, L, Na, Nb, 2)
    gt = np.transpose(g, (0, 2, 1))
    assert np.abs(_align(gt, ref) - ref).max() > 1e-3
