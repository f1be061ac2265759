"""Pins of the oracle's DMRG-RPA (Sec. II C eq. dmrgrpa, Sec. II D, Sec. III E
eqs. reducedrpa and bmatrix) against results fixed independently of its
construction of the second-order vectors:

* the second variation of the energy on the MPS manifold: at a stationary
  reference, for any curve Psi(eps) through it, d^2E/d eps^2 / 2 =
  x^T (A + W) x, x the tangent coordinates of dPsi/d eps, i.e.
  x^T W x = 2 <Psi_2 | (H - E0) Psi0>, Psi_2 the eps^2 coefficient.  The
  curve perturbs every site tensor of a mixed-canonical representation at
  once and its coefficients come from a polynomial fit of the FCI vectors
  (no projectors, no Lambda, no split into left and right pieces);
* an exact reference (full bond dimension): W = 0 and the RPA roots are the
  TDA roots, which are the FCI excitation energies;
* at a stable stationary reference: the roots come in +-omega pairs, omega^2
  are the eigenvalues of (A - W)(A + W) (the textbook reduction), and the
  lowest RPA root lies below the lowest TDA root (Thouless' variational
  bound: the TDA vector is a trial vector of the RPA functional);
* a planted mistake (Lambda^-1 dropped from the first-order left tensor)
  breaks the second-variation identity;
* the two sweep directions of eq. bmatrix (pairs grouped by their right site
  with first-order left block states, or by their left site with
  first-order right block states) give the same W;
* at a stationary reference the site-wise W gradient of the library's RPA
  residual is the exact one (P_i^T of the representer of W(., v)).
"""
import numpy as np
import pytest

import synth
from oracle import fci, firstorder, mpsvec, response, rpa, tda


def _reference(L, Na, Nb, M, seed, stable_shift=True):
    h, eri, ecore = synth.random_integrals(L, seed=seed, K=L, diag_lo=-2, diag_hi=0)
    dets, H = fci.hamiltonian(h, eri, ecore, Na, Nb)
    mps = synth.random_mps(L, Na, Nb, M, seed)
    Hs = rpa.stationary_hamiltonian(mps, dets, H)
    psi0 = mpsvec.mps_to_fci(mps, dets)
    psi0 /= np.linalg.norm(psi0)
    if stable_shift:
        # lift every direction orthogonal to Psi0: A grows by lam, (H - E0) Psi0
        # and hence W are unchanged; lam makes A +- W positive definite
        e0, A, W, _ = rpa.rpa_matrices(mps, dets, Hs)
        lam = 1.0 + 2.0 * (np.linalg.norm(W, 2) + max(0.0, -np.linalg.eigvalsh(A).min()))
        Hs = Hs + lam * (np.eye(len(dets)) - np.outer(psi0, psi0))
    return mps, dets, Hs, psi0


def _curve_coefficients(mps, dets, c, delta):
    """FCI-vector coefficients Psi_k of Psi(eps) = MPS(T + eps delta), T the
    mixed-canonical tensors L_0..L_{c-1} C_c R_{c+1}.. (a polynomial of degree
    L in eps), by a fit on L+1 Chebyshev nodes."""
    L = mps.L
    base = [mps.Lt[i] if i < c else (mps.Ct[i] if i == c else mps.Rt[i]) for i in range(L)]
    nodes = 0.5 * np.cos(np.pi * (np.arange(L + 1) + 0.5) / (L + 1))
    vals = []
    for e in nodes:
        T = [{k: base[i][k] + e * delta[i][k] for k in base[i]} for i in range(L)]
        vals.append(firstorder.fci_vector(mps, dets, T, T[c], T, c))
    V = np.vander(nodes, L + 1, increasing=True)
    return np.linalg.solve(V, np.array(vals))


def _random_delta(mps, rng):
    return [{k: rng.normal(size=b.shape) for k, b in mps.Ct[i].items()} for i in range(mps.L)]


def _second_variation_errors(mps, dets, Hs, psi0, ndir, seed):
    e0, A, W, B = rpa.rpa_matrices(mps, dets, Hs)
    h0 = Hs @ psi0 - e0 * psi0
    rng = np.random.default_rng(seed)
    errs = []
    for k in range(ndir):
        c = [0, mps.L // 2, mps.L - 1][k % 3]
        coef = _curve_coefficients(mps, dets, c, _random_delta(mps, rng))
        assert np.linalg.norm(coef[0] - psi0) < 1e-10
        x = B.T @ coef[1]
        # dPsi/d eps lies in the tangent space (plus a Psi0 component)
        resid = coef[1] - psi0 * (psi0 @ coef[1]) - B @ x
        assert np.linalg.norm(resid) < 1e-9 * np.linalg.norm(coef[1])
        lhs = x @ W @ x
        rhs = 2.0 * coef[2] @ h0
        errs.append(abs(lhs - rhs) / max(1.0, abs(rhs), np.linalg.norm(x) ** 2 * np.linalg.norm(h0)))
    return errs


@pytest.mark.parametrize("L,Na,Nb,M,seed", [(4, 2, 2, 4, 3), (5, 2, 2, 6, 11), (5, 3, 2, 5, 17)])
def test_w_is_the_second_variation_at_a_stationary_reference(L, Na, Nb, M, seed):
    mps, dets, Hs, psi0 = _reference(L, Na, Nb, M, seed, stable_shift=False)
    # the reference is stationary: (H - E0) Psi0 has no tangent component
    T, _ = tda.tangent_basis(mps, dets)
    e0 = float(psi0 @ Hs @ psi0)
    g = T.T @ (Hs @ psi0 - e0 * psi0)
    assert np.linalg.norm(g) < 1e-11
    # and W is not trivially zero there
    _, _, W, _ = rpa.rpa_matrices(mps, dets, Hs)
    assert np.abs(W).max() > 1e-3
    errs = _second_variation_errors(mps, dets, Hs, psi0, 3, seed)
    assert max(errs) < 1e-9, errs


def test_planted_missing_lambda_inverse_breaks_the_second_variation(monkeypatch):
    mps, dets, Hs, psi0 = _reference(5, 2, 2, 6, 11, stable_shift=False)

    def identity_gauge(m, i):
        return {c: np.eye(g.shape[0]) for c, g in rpa.__dict__["_true_gauge"](m, i).items()}

    monkeypatch.setitem(rpa.__dict__, "_true_gauge", rpa.gauge_matrix)
    monkeypatch.setattr(rpa, "gauge_matrix", identity_gauge)
    errs = _second_variation_errors(mps, dets, Hs, psi0, 2, 5)
    assert max(errs) > 1e-4, errs


def test_exact_reference_rpa_equals_tda_equals_fci():
    L, Na, Nb = 5, 2, 2
    h, eri, ecore = synth.random_integrals(L, seed=31, K=5, diag_lo=-2, diag_hi=0)
    dets, H, w, vec = fci.fci(h, eri, ecore, Na, Nb, nroots=6)
    bonds, A = mpsvec.fci_to_mps(vec[:, 0], dets, L, Na, Nb)
    mps = synth.canonical_from_tensors(L, Na, Nb, bonds, A)
    e0, Am, W, _ = rpa.rpa_matrices(mps, dets, H)
    assert np.abs(W).max() < 1e-9
    e0, om_rpa, om_tda = rpa.rpa_roots(mps, dets, H, 5)
    np.testing.assert_allclose(om_rpa, om_tda, atol=1e-9)
    np.testing.assert_allclose(om_tda, w[1:6] - w[0], atol=1e-9)


@pytest.mark.parametrize("L,Na,Nb,M,seed", [(5, 2, 2, 6, 11), (6, 3, 3, 8, 23)])
def test_stable_stationary_reference_rpa_properties(L, Na, Nb, M, seed):
    mps, dets, Hs, psi0 = _reference(L, Na, Nb, M, seed)
    e0, A, W, _ = rpa.rpa_matrices(mps, dets, Hs)
    np.testing.assert_allclose(W, W.T, atol=1e-12 * max(1.0, np.abs(W).max()))
    assert np.linalg.eigvalsh(A + W).min() > 0 and np.linalg.eigvalsh(A - W).min() > 0
    n = A.shape[0]
    full = np.sort(np.linalg.eigvals(np.block([[A, W], [-W, -A]])).real)
    np.testing.assert_allclose(full[:n], -full[n:][::-1], atol=1e-9 * full.max())
    om = rpa.rpa_solve(A, W)
    assert om.min() > 0
    w2 = np.sort(np.linalg.eigvals((A - W) @ (A + W)).real)
    np.testing.assert_allclose(om ** 2, w2, rtol=1e-9, atol=1e-9 * w2.max())
    tda_w = np.linalg.eigvalsh(A)
    assert om[0] <= tda_w[0] + 1e-12
    # W is not negligible here, so the bound is strict
    assert om[0] < tda_w[0] - 1e-6


def _project_right(mps, dets, Rt, site, v):
    """Components of v along |l n r'> at `site`, the right states r' built
    from the tensors Rt[site+1..] (left states from the MPS's L tensors)."""
    left = mpsvec._left_states(mps, mps.Lt, site)
    right = mpsvec._right_states(mps, Rt, site + 1)
    out = []
    for a, n, c in mps.block_keys(site):
        ml, mr = mps.bonds[site][a][1], mps.bonds[site + 1][c][1]
        if a in left and c in right:
            cl, Ul = left[a]
            cr, Ur = right[c]
            pos = np.searchsorted(dets, (cl[:, None] | (np.int64(n) << (2 * site)) | cr[None, :]).ravel())
            out.append((Ul.T @ v[pos].reshape(len(cl), len(cr)) @ Ur).ravel())
        else:
            out.append(np.zeros(ml * mr))
    return np.concatenate(out)


def test_backward_sweep_form_of_the_w_matrix_equals_the_forward_form():
    # eq. bmatrix accumulates W over the sites of one sweep.  The oracle
    # groups each pair (p < q) by its right site q: the first-order left
    # states of x up to q-1 and the right-gauge piece of y at q.  The library's
    # backward sweep groups it by its left site p: the left-gauge piece of x
    # at p and the first-order right states of y beyond p, built from
    # R1_q = Lambda_{q-1}^-1 (C_q Q^R).  Both must give the same matrix.
    L, Na, Nb, M, seed = 5, 2, 2, 6, 11
    mps, dets, Hs, psi0 = _reference(L, Na, Nb, M, seed, stable_shift=False)
    e0, A, W, B = rpa.rpa_matrices(mps, dets, Hs)
    h0 = Hs @ psi0 - e0 * psi0
    lam_inv = [{c: np.linalg.inv(g) for c, g in rpa.gauge_matrix(mps, i).items()} for i in range(L - 1)]
    nb = B.shape[1]
    pieces = [rpa.site_pieces(mps, dets, B[:, a]) for a in range(nb)]
    left_flat = [np.stack([firstorder.flat(mps, p, pieces[a][0][p]) for a in range(nb)]) for p in range(L)]
    half = np.zeros((nb, nb))
    for b in range(nb):
        br = pieces[b][1]
        # R1_q[b] = Lambda_{q-1}^-1 (C_q Q^R), Lambda keyed by the left sector of site q
        r1 = [None] + [{(s, n): lam_inv[q - 1][s] @ blk for (s, n), blk in br[q].items()} for q in range(1, L)]
        for p in range(L - 1):
            gam = np.zeros(mps.site_size(p))
            for q in range(p + 1, L):
                Rt = list(mps.Rt)
                Rt[q] = r1[q]
                gam += _project_right(mps, dets, Rt, p, h0)
            half[:, b] += left_flat[p] @ gam
    np.testing.assert_allclose(half + half.T, W, atol=1e-12 * max(1.0, np.abs(W).max()))


@pytest.mark.parametrize("L,Na,Nb,M,seed", [(4, 2, 2, 4, 3), (5, 2, 2, 6, 11), (5, 3, 2, 5, 17)])
def test_site_gradient_of_w_at_a_stationary_reference(L, Na, Nb, M, seed):
    # The DMRG-RPA residual takes the site-i part of W v from the mixed-
    # canonical MPS centred at i: <U_v n r|H|Psi0> + <l n V_v|H|Psi0>, with
    # U_v (V_v) the first-order left (right) block states of v, projected off
    # C^(0).  At a stationary reference that is exactly P_i^T w_v, where
    # w_v = B W B^T v is the tangent-space representer of W(., v).
    mps, dets, Hs, psi0 = _reference(L, Na, Nb, M, seed, stable_shift=False)
    e0, A, W, B = rpa.rpa_matrices(mps, dets, Hs)
    h0 = Hs @ psi0 - e0 * psi0
    lam_inv = [{c: np.linalg.inv(g) for c, g in rpa.gauge_matrix(mps, i).items()} for i in range(L - 1)]
    C0 = [firstorder.site_project(mps, dets, i, psi0) for i in range(L)]
    rng = np.random.default_rng(seed)
    for _ in range(2):
        c = rng.normal(size=B.shape[1])
        v, wv = B @ c, B @ (W @ c)
        bl, br = rpa.site_pieces(mps, dets, v)
        l1 = [{(s, n): b @ lam_inv[p][firstorder._right_sector(mps, p, s, n)] for (s, n), b in bl[p].items()}
              for p in range(L - 1)]
        r1 = [None] + [{(a, n): lam_inv[q - 1][a] @ b for (a, n), b in br[q].items()} for q in range(1, L)]
        for i in range(L):
            g = np.zeros(mps.site_size(i))
            for p in range(i):
                Lt = list(mps.Lt)
                Lt[p] = l1[p]
                g += rpa._project(mps, dets, Lt, i, h0)
            for q in range(i + 1, L):
                Rt = list(mps.Rt)
                Rt[q] = r1[q]
                g += _project_right(mps, dets, Rt, i, h0)
            g -= C0[i] * (C0[i] @ g)
            exact = firstorder.site_project(mps, dets, i, wv)
            assert np.linalg.norm(g - exact) <= 1e-11 * max(1.0, np.linalg.norm(exact)), (i, np.linalg.norm(g - exact))
