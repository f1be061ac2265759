"""Pins of the FP64 CPU oracle against closed forms, brute force and exact
results (no GPU).  Each test states what fixes the expected value."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import fci, fock, mpsvec, tda


def test_determinant_count_config0():
    # 8 orbitals, 4 alpha + 4 beta electrons: C(8,4)^2 determinants
    assert len(fci.determinants(8, 4, 4)) == 4900 == math.comb(8, 4) ** 2


@pytest.mark.parametrize("L,Na,Nb", [(2, 1, 1), (3, 2, 1), (3, 1, 2)])
def test_fci_matches_bruteforce_fock_space(L, Na, Nb):
    # Independent construction: literal products of Jordan-Wigner matrices.
    h, eri, _ = synth.random_integrals(L, seed=7 + L + Na, K=4, diag_lo=-1, diag_hi=0.5)
    dets, H = fci.hamiltonian(h, eri, 0.3, Na, Nb)
    Hf = fock.fock_hamiltonian(h, eri, 0.3)
    idx = fock.sector_indices(L, Na, Nb)
    assert np.array_equal(np.sort(idx), dets)
    np.testing.assert_allclose(H.toarray(), Hf[np.ix_(dets, dets)], atol=1e-12)


def test_one_body_spectrum_is_sums_of_orbital_energies():
    # Without two-electron integrals every eigenstate is a determinant of
    # the eigenorbitals of h: the spectrum is all sums of Na + Nb orbital energies.
    L, Na, Nb = 5, 2, 2
    h, _, _ = synth.random_integrals(L, seed=3, K=1, diag_lo=-2, diag_hi=0)
    eri = np.zeros((L,) * 4)
    dets, H = fci.hamiltonian(h, eri, 0.0, Na, Nb)
    w = np.linalg.eigvalsh(H.toarray())
    eps = np.linalg.eigvalsh(h)
    sums = sorted(sum(eps[list(a)]) + sum(eps[list(b)])
                  for a in itertools.combinations(range(L), Na)
                  for b in itertools.combinations(range(L), Nb))
    np.testing.assert_allclose(w, sums, atol=1e-12)


@pytest.mark.parametrize("t,U", [(1.0, 4.0), (0.5, 1.3), (2.0, 0.0)])
def test_hubbard_dimer_closed_form(t, U):
    # Two sites, one alpha and one beta electron: E0 = (U - sqrt(U^2 + 16 t^2)) / 2
    h = np.array([[0.0, -t], [-t, 0.0]])
    eri = np.zeros((2,) * 4)
    eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
    _, _, w, _ = fci.fci(h, eri, 0.0, 1, 1, nroots=1)
    assert abs(w[0] - (U - math.sqrt(U * U + 16 * t * t)) / 2) < 1e-12


def test_two_body_normalization_constant_interaction():
    # (ij|kl) = c d_ij d_kl makes the two-electron operator c/2 (N^2 - N).
    L, Na, Nb, c = 4, 2, 1, 0.37
    eri = np.zeros((L,) * 4)
    for i in range(L):
        for k in range(L):
            eri[i, i, k, k] = c
    dets, H = fci.hamiltonian(np.zeros((L, L)), eri, 0.0, Na, Nb)
    N = Na + Nb
    np.testing.assert_allclose(H.toarray(), c / 2 * (N * N - N) * np.eye(len(dets)), atol=1e-13)


def _small_problem(L=6, Na=3, Nb=3, seed=11):
    h, eri, e0 = synth.random_integrals(L, seed=seed, K=6, diag_lo=-2, diag_hi=0)
    return h, eri, e0, Na, Nb


def test_mps_vector_independent_of_center():
    h, eri, e0, Na, Nb = _small_problem()
    mps = synth.random_mps(6, Na, Nb, 12, seed=5)
    dets = fci.determinants(6, Na, Nb)
    ref = mpsvec.mps_to_fci(mps, dets)
    assert abs(np.linalg.norm(ref) - 1) < 1e-12
    for i in range(6):
        np.testing.assert_allclose(mpsvec.mps_to_fci(mps, dets, site=i), ref, atol=1e-12)


def test_site_basis_orthonormal_and_energy_gauge_invariant():
    h, eri, e0, Na, Nb = _small_problem()
    mps = synth.random_mps(6, Na, Nb, 12, seed=6)
    dets, H = fci.hamiltonian(h, eri, e0, Na, Nb)
    psi = mpsvec.mps_to_fci(mps, dets)
    E = mpsvec.energy(H, psi)
    for i in range(6):
        P = mpsvec.site_basis(mps, dets, i)
        np.testing.assert_allclose(P.T @ P, np.eye(P.shape[1]), atol=1e-12)
        c = mps.flat("C", i)
        np.testing.assert_allclose(P @ c, psi, atol=1e-12)
        He = mpsvec.heff(H, P)
        assert abs(c @ He @ c - E) < 1e-11


def test_heff_full_space_has_fci_spectrum():
    # With untruncated bonds the product basis is complete, so H_eff is H in
    # another orthonormal basis (same spectrum), one-site and two-site.
    L, Na, Nb = 5, 2, 3
    h, eri, e0 = synth.random_integrals(L, seed=21, K=5, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, 10 ** 6, seed=2)
    dets, H = fci.hamiltonian(h, eri, e0, Na, Nb)
    w = np.linalg.eigvalsh(H.toarray())
    P = mpsvec.site_basis(mps, dets, 2)
    assert P.shape == (len(dets), len(dets))
    np.testing.assert_allclose(np.linalg.eigvalsh(mpsvec.heff(H, P)), w, atol=1e-11)
    P2 = mpsvec.two_site_basis(mps, dets, 1)
    np.testing.assert_allclose(np.linalg.eigvalsh(mpsvec.heff(H, P2)), w, atol=1e-11)


def test_tangent_space_rank_equals_nonredundant_count():
    # Parameters minus one GL(m_q) gauge per internal bond sector (injective MPS).
    mps = synth.random_mps(6, 3, 3, 10, seed=9)
    dets = fci.determinants(6, 3, 3)
    _, rank = tda.tangent_basis(mps, dets)
    assert rank == tda.redundancy_free_rank(mps)


def test_tda_exact_on_exact_ground_state():
    # With the exact ground state as reference and untruncated bonds the
    # tangent space is the whole sector, so the TDA roots are the FCI
    # excited-state energies (formal exactness as M -> infinity).
    L, Na, Nb = 5, 2, 2
    h, eri, e0 = synth.random_integrals(L, seed=31, K=5, diag_lo=-2, diag_hi=0)
    dets, H, w, v = fci.fci(h, eri, e0, Na, Nb, nroots=6)
    bonds, A = mpsvec.fci_to_mps(v[:, 0], dets, L, Na, Nb)
    mps = synth.canonical_from_tensors(L, Na, Nb, bonds, A)
    psi = mpsvec.mps_to_fci(mps, dets)
    assert abs(abs(psi @ v[:, 0]) - 1) < 1e-12
    E0, roots = tda.tda_roots(mps, dets, H, 5)
    assert abs(E0 - w[0]) < 1e-11
    np.testing.assert_allclose(roots, w[1:6], atol=1e-10)


def test_matrix_free_heff_apply_equals_explicit_heff():
    # P^T H P c evaluated block by block (no P formed) equals the explicit
    # product with P from the column construction, one- and two-site; at the
    # full space the matrix-free map reproduces H's spectrum on its own.
    h, eri, e0, Na, Nb = _small_problem()
    mps = synth.random_mps(6, Na, Nb, 12, seed=8)
    dets, H = fci.hamiltonian(h, eri, e0, Na, Nb)
    rng = np.random.default_rng(3)
    for i in range(6):
        P = mpsvec.site_basis(mps, dets, i)
        C = rng.normal(size=(2, P.shape[1]))
        np.testing.assert_allclose(mpsvec.heff_apply(H, mps, dets, i, C), C @ mpsvec.heff(H, P).T, atol=1e-12)
    for i in range(5):
        P = mpsvec.two_site_basis(mps, dets, i)
        C = rng.normal(size=(2, P.shape[1]))
        np.testing.assert_allclose(mpsvec.heff_apply(H, mps, dets, i, C, width=2), C @ mpsvec.heff(H, P).T,
                                   atol=1e-12)
    L, Na, Nb = 4, 2, 2
    h, eri, e0 = synth.random_integrals(L, seed=22, K=4, diag_lo=-2, diag_hi=0)
    full = synth.random_mps(L, Na, Nb, 10 ** 6, seed=4)
    dets, H = fci.hamiltonian(h, eri, e0, Na, Nb)
    n = full.site_size(1)
    assert n == len(dets)
    He = mpsvec.heff_apply(H, full, dets, 1, np.eye(n))
    np.testing.assert_allclose(np.linalg.eigvalsh(He), np.linalg.eigvalsh(H.toarray()), atol=1e-11)


def test_fci_refuses_spaces_above_the_dense_limit():
    # L=9, 4+4 electrons: 126^2 = 15876 determinants, above the dense limit
    L = 9
    h, eri, _ = synth.random_integrals(L, seed=1, K=2, diag_lo=-1, diag_hi=0)
    with pytest.raises(ValueError):
        fci.fci(h, eri, 0.0, 4, 4)
