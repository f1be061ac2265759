"""Pins of the oracle's first-order wavefunctions and TDA sigma
(oracle/firstorder.py) on the CPU, each against something other than its
own formula:

* the gauge projections give tensors that satisfy the gauge conditions of
  Sec. II B (eqs. left-orthoSeb, right-orthoSeb) and leave the first-order
  components orthogonal to the reference state (computed by
  mpsvec.mps_to_fci, pinned in test_oracle);
* each first-order component is the derivative of the MPS wavefunction
  along that tensor (Sec. II B, eq. psi1st): the wavefunction is linear in
  each site tensor, so the difference of two MPS wavefunctions built by
  mpsvec.mps_to_fci equals the component exactly;
* the first-order wavefunction lies in the tangent space spanned by the
  one-site product bases (oracle.tda.tangent_basis);
* the site projection equals the explicit product with the pinned P_i, and
  the TDA sigma with only a centre component reduces to the explicit
  effective Hamiltonian (Sec. III D: H_0^[i] C^(1))."""
import copy

import numpy as np
import pytest

import synth
from oracle import fci, firstorder, mpsvec, tda


@pytest.fixture(scope="module")
def small():
    L, Na, Nb, M = 6, 3, 2, 10
    h, eri, _ = synth.random_integrals(L, seed=41, K=6, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, M, seed=42)
    dets, H = fci.hamiltonian(h, eri, 0.2, Na, Nb)
    return L, mps, dets, H


def _rand(mps, i, rng):
    return firstorder.blocks(mps, i, rng.normal(size=mps.site_size(i)))


def test_flat_blocks_round_trip(small):
    L, mps, dets, H = small
    x = np.random.default_rng(0).normal(size=mps.site_size(2))
    np.testing.assert_array_equal(firstorder.flat(mps, 2, firstorder.blocks(mps, 2, x)), x)
    np.testing.assert_array_equal(firstorder.flat(mps, 3, mps.Ct[3]), mps.flat("C", 3))


def test_gauge_projections_satisfy_gauge_conditions(small):
    L, mps, dets, H = small
    rng = np.random.default_rng(1)
    for i in range(L):
        X = _rand(mps, i, rng)
        QL = firstorder.q_left(mps, i, X)
        XQ = firstorder.q_right(mps, i, X)
        # sum over (l, n) of L^T L1 vanishes per right sector; sum over (n, r)
        # of R1 R^T per left sector (left-orthoSeb / right-orthoSeb)
        right = mps.sector_index(i + 1)
        for c in range(len(right)):
            g = sum(mps.Lt[i][(a, n)].T @ QL[(a, n)] for a, n, cc in mps.block_keys(i) if cc == c)
            if not np.isscalar(g):
                assert np.abs(g).max() < 1e-12
        for a in range(len(mps.bonds[i])):
            g = sum(XQ[(aa, n)] @ mps.Rt[i][(aa, n)].T for aa, n, _ in mps.block_keys(i) if aa == a)
            if not np.isscalar(g):
                assert np.abs(g).max() < 1e-12
        # projectors: idempotent, and they annihilate the zeroth-order tensor
        Q2 = firstorder.q_left(mps, i, QL)
        assert max(np.abs(Q2[k] - QL[k]).max() for k in QL) < 1e-12
        ZL = firstorder.q_left(mps, i, mps.Lt[i])
        ZR = firstorder.q_right(mps, i, mps.Rt[i])
        assert max(np.abs(v).max() for v in ZL.values()) < 1e-12
        assert max(np.abs(v).max() for v in ZR.values()) < 1e-12


@pytest.mark.parametrize("i", [1, 3, 5])
def test_components_are_derivatives_of_the_mps(small, i):
    L, mps, dets, H = small
    rng = np.random.default_rng(10 + i)
    psi0 = mpsvec.mps_to_fci(mps, dets, site=i)
    for j in range(L):
        X = _rand(mps, j, rng)
        if j < i:
            comp = firstorder.first_order_psi(mps, dets, i, {j: X}, None, {})
            P = firstorder.q_left(mps, j, X)
            pert = copy.copy(mps)
            pert.Lt = list(mps.Lt)
            pert.Lt[j] = {k: mps.Lt[j][k] + P[k] for k in P}
        elif j == i:
            comp = firstorder.first_order_psi(mps, dets, i, {}, X, {})
            pert = copy.copy(mps)
            pert.Ct = list(mps.Ct)
            pert.Ct[i] = {k: mps.Ct[i][k] + X[k] for k in X}
        else:
            comp = firstorder.first_order_psi(mps, dets, i, {}, None, {j: X})
            P = firstorder.q_right(mps, j, X)
            pert = copy.copy(mps)
            pert.Rt = list(mps.Rt)
            pert.Rt[j] = {k: mps.Rt[j][k] + P[k] for k in P}
        diff = mpsvec.mps_to_fci(pert, dets, site=i) - psi0
        assert np.abs(diff - comp).max() < 1e-12, j
        if j != i:
            # the gauge conditions make the component orthogonal to Psi0
            assert abs(comp @ psi0) < 1e-12, j


def test_first_order_psi_lies_in_tangent_space(small):
    L, mps, dets, H = small
    rng = np.random.default_rng(3)
    i = 2
    L1 = {j: _rand(mps, j, rng) for j in range(i)}
    R1 = {j: _rand(mps, j, rng) for j in range(i + 1, L)}
    psi1 = firstorder.first_order_psi(mps, dets, i, L1, _rand(mps, i, rng), R1)
    Q, _ = tda.tangent_basis(mps, dets)
    assert np.linalg.norm(psi1 - Q @ (Q.T @ psi1)) < 1e-10 * np.linalg.norm(psi1)


def test_site_projection_and_centre_term(small):
    L, mps, dets, H = small
    rng = np.random.default_rng(4)
    for i in (0, 3, L - 1):
        v = rng.normal(size=len(dets))
        P = mpsvec.site_basis(mps, dets, i)
        np.testing.assert_allclose(firstorder.site_project(mps, dets, i, v), P.T @ v, atol=1e-12)
        c1 = rng.normal(size=mps.site_size(i))
        sig = firstorder.tda_sigma(H, mps, dets, i, {}, firstorder.blocks(mps, i, c1), {})
        np.testing.assert_allclose(sig, mpsvec.heff(H, P) @ c1, atol=1e-11)


def test_left_part_is_linear_in_the_centre(small):
    # the first line of eq. sigv2 applied to C_i^(0) equals the left part of
    # the full TDA sigma without centre and right components
    L, mps, dets, H = small
    rng = np.random.default_rng(5)
    i = 4
    L1 = {j: _rand(mps, j, rng) for j in range(i)}
    a = firstorder.dh_left(H, mps, dets, i, L1, mps.Ct[i])
    b = firstorder.tda_sigma(H, mps, dets, i, L1, None, {})
    np.testing.assert_allclose(a, b, atol=1e-12)
