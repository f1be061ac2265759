"""Pins of the oracle's tangent-space linear response (Sec. II B, eqs.
realresp and imagresp) against results fixed independently of it: the
exact sum over FCI states when the tangent space is the whole sector, the
spectral decomposition of the projected Hamiltonian, the one-body operator
against second quantization in Fock space, and the symmetries of the two
frequency components."""
import numpy as np
import pytest

import synth
from oracle import fci, fock, mpsvec, response, tda


def _random_v(L, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(L, L))
    return 0.5 * (v + v.T)


def test_onebody_matrix_matches_fock_space_operator():
    # V = sum_pq v_pq (a+_pa a_qa + a+_pb a_qb) built in the full Fock space
    # from creation / annihilation matrices, restricted to the sector
    L, Na, Nb = 3, 2, 1
    v = _random_v(L, 1)
    dets, _ = fci.hamiltonian(v, np.zeros((L,) * 4), 0.0, Na, Nb)
    F = fock.fock_hamiltonian(v, np.zeros((L,) * 4), 0.0)
    idx = fock.sector_indices(L, Na, Nb)
    Fs = F[np.ix_(idx, idx)]
    V = response.onebody(v, Na, Nb)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(V)), np.sort(np.linalg.eigvalsh(Fs)), atol=1e-12)


def test_exact_reference_gives_the_fci_sum_over_states():
    # exact ground state at full bond dimension: the tangent space is the
    # whole orthogonal complement of Psi0, so chi_pm is the textbook
    # -sum_{n>0} |<n|V|0>|^2 / (E_n - E0 +- omega) over FCI eigenstates
    L, Na, Nb = 5, 2, 2
    h, eri, e0 = synth.random_integrals(L, seed=31, K=5, diag_lo=-2, diag_hi=0)
    dets, H, w, vec = fci.fci(h, eri, e0, Na, Nb, nroots=len(fci.determinants(L, Na, Nb)))
    bonds, A = mpsvec.fci_to_mps(vec[:, 0], dets, L, Na, Nb)
    mps = synth.canonical_from_tensors(L, Na, Nb, bonds, A)
    V = response.onebody(_random_v(L, 7), Na, Nb)
    W, U = np.linalg.eigh(H.toarray())
    t = (U[:, 1:].T @ (V @ U[:, 0])) ** 2
    for omega in (0.0, 0.05, 0.2):
        cp, cm = response.response(mps, dets, H, V, omega)
        ref_p = -np.sum(t / (W[1:] - W[0] + omega))
        ref_m = -np.sum(t / (W[1:] - W[0] - omega))
        assert abs(cp - ref_p) < 1e-9 * max(1.0, abs(ref_p)), (omega, cp, ref_p)
        assert abs(cm - ref_m) < 1e-9 * max(1.0, abs(ref_m)), (omega, cm, ref_m)
    # the static response of the ground state is negative (H - E0 > 0 on the complement)
    cp, cm = response.response(mps, dets, H, V, 0.0)
    assert cp < 0 and abs(cp - cm) < 1e-12 * abs(cp)


def test_truncated_reference_is_the_tangent_spectral_sum():
    # truncated random MPS: the same chi from the eigenpairs of the projected
    # Hamiltonian (a different route than the linear solve), and
    # chi_+(omega) = chi_-(-omega)
    L, Na, Nb, M = 6, 3, 3, 12
    h, eri, e0 = synth.random_integrals(L, seed=11, K=6, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, M, seed=12)
    dets, H = fci.hamiltonian(h, eri, e0, Na, Nb)
    V = response.onebody(_random_v(L, 3), Na, Nb)
    psi0, B = response.tangent_space(mps, dets)
    E0 = float(psi0 @ (H @ psi0))
    ek, uk = np.linalg.eigh(B.T @ (H @ B))
    bk = uk.T @ (B.T @ (V @ psi0))
    # its dimension is the TDA's (same space)
    assert B.shape[1] == tda.tangent_basis(mps, dets)[1] - 1
    for omega in (0.1, 0.37):
        cp, cm = response.response(mps, dets, H, V, omega)
        assert abs(cp + np.sum(bk ** 2 / (ek - (E0 - omega)))) < 1e-9 * max(1.0, abs(cp))
        assert abs(cm + np.sum(bk ** 2 / (ek - (E0 + omega)))) < 1e-9 * max(1.0, abs(cm))
        cp2, cm2 = response.response(mps, dets, H, V, -omega)
        assert abs(cp - cm2) < 1e-10 * max(1.0, abs(cp)) and abs(cm - cp2) < 1e-10 * max(1.0, abs(cm))


def test_planted_sign_error_in_the_shift_is_caught():
    # a mistake in the oracle (shift E0 + omega where E0 - omega belongs)
    # breaks the sum-over-states pin at nonzero omega
    L, Na, Nb = 4, 2, 2
    h, eri, e0 = synth.random_integrals(L, seed=5, K=4, diag_lo=-2, diag_hi=0)
    dets, H, w, vec = fci.fci(h, eri, e0, Na, Nb, nroots=len(fci.determinants(L, Na, Nb)))
    bonds, A = mpsvec.fci_to_mps(vec[:, 0], dets, L, Na, Nb)
    mps = synth.canonical_from_tensors(L, Na, Nb, bonds, A)
    V = response.onebody(_random_v(L, 9), Na, Nb)
    W, U = np.linalg.eigh(H.toarray())
    t = (U[:, 1:].T @ (V @ U[:, 0])) ** 2
    omega = 0.15
    _, cm = response.response(mps, dets, H, V, omega)   # shift E0 + omega
    ref_p = -np.sum(t / (W[1:] - W[0] + omega))
    assert abs(cm - ref_p) > 1e-6
