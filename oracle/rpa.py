"""DMRG-RPA of an MPS reference in its tangent space (oracle; test
infrastructure only).

Definitions followed:
  * Sec. II C, eq. dmrgrpa: the RPA problem
        [[H, W], [W*, H*]] (X, Y) = omega [[S, 0], [0, -S*]] (X, Y)
    with H_ij = <d_i Psi0 | H - E0 | d_j Psi0>, S_ij = <d_i Psi0 | d_j Psi0>
    and W_ij = <d_i d_j Psi0 | H - E0 | Psi0>, the first derivatives taken
    orthogonal to Psi0 (Q^(1)) and the second ones orthogonal to the
    first-order space and Psi0 (Q^(2)).  Everything here is real, so W* = W.
    In an orthonormal basis B of the tangent space with Psi0 removed (the
    TDA oracle's space) S = 1 and H is B^T (H - E0) B.
  * Sec. II D (non-redundant parameterization): for sites p < q the
    second-order vectors are built in the mixed-canonical gauge centred
    between p and q, with the first-order left tensor at p and the
    first-order right tensor at q:
        Phi_pq[x, y] = L_0..L_{p-1} L1_p[x] L_{p+1}..L_{q-1} Lambda_{q-1} R1_q[y] R_{q+1}..
    (for q = p + 1 this is L1_p Lambda_p R1_{p+1}, the paper's nearest-
    neighbour example).  L1_p[x] = (Q^L G_p[x]) Lambda_p^{-1} (eq. left1st) and
    Lambda_{q-1} R1_q[y] = G_q[y] Q^R (eq. right1st), where G_i[v] is the
    site-i centre tensor of the first-order vector v: its projection on the
    one-site product basis of site i (eqs. gauge_fwd, gauge_bwd).  Lambda_i
    is L_i^T C_i (the gauge matrix of the shift between sites i and i+1).
    The second derivative along (x, y) is the sum over p < q of
    Phi_pq[x, y] + Phi_pq[y, x], so
        W(x, y) = sum_{p<q} <Phi_pq[x, y] + Phi_pq[y, x] | (H - E0) Psi0>.
    Grouping the left factors of one q gives eq. bmatrix: the first-order
    left block states of x at bond q-1, the right-gauge piece of y at q.
  * Sec. III E, eq. reducedrpa: the RPA roots are the positive eigenvalues
    of [[A, W], [-W, -A]] (the metric diag(1, -1) moved to the left), A the
    TDA matrix; they come in pairs +-omega.

W is evaluated column by column: for each basis vector x and each q the
projection of (H - E0) Psi0 on the product basis of site q with the left
states replaced by the first-order ones of x (all p < q summed) is formed
once, and dotted with the right-gauge pieces of every y.
"""
from __future__ import annotations

import numpy as np

from . import firstorder, mpsvec, response, tda

QN = firstorder.QN


def gauge_matrix(mps, i):
    """Lambda_i = L_i^T C_i per right sector c at bond i+1 (the gauge
    matrix of the shift between sites i and i+1)."""
    out = {}
    for (a, n), Lb in mps.Lt[i].items():
        c = firstorder._right_sector(mps, i, a, n)
        g = Lb.T @ mps.Ct[i][(a, n)]
        out[c] = out[c] + g if c in out else g
    return out


def site_pieces(mps, dets, v):
    """Left- and right-gauge pieces (Q^L G_i, G_i Q^R) at every site of a
    tangent-space FCI vector v, G_i its site-i centre tensor."""
    bl, br = [], []
    for i in range(mps.L):
        G = firstorder.blocks(mps, i, firstorder.site_project(mps, dets, i, v))
        bl.append(firstorder.q_left(mps, i, G))
        br.append(firstorder.q_right(mps, i, G))
    return bl, br


def _project(mps, dets, Lt, site, v):
    """Components of the FCI vector v along the product basis |l n r> of
    site `site` whose left states are built from the tensors Lt[0..site-1]
    (right states from the MPS's R tensors); flat, library block order."""
    left = mpsvec._left_states(mps, Lt, site)
    right = mpsvec._right_states(mps, mps.Rt, site + 1)
    out = []
    for a, n, c in mps.block_keys(site):
        ml, mr = mps.bonds[site][a][1], mps.bonds[site + 1][c][1]
        if a in left and c in right:
            cl, Ul = left[a]
            cr, Ur = right[c]
            cfg = (cl[:, None] | (np.int64(n) << (2 * site)) | cr[None, :]).ravel()
            pos = np.searchsorted(dets, cfg)
            assert (dets[np.minimum(pos, len(dets) - 1)] == cfg).all(), "configuration outside the sector"
            out.append((Ul.T @ v[pos].reshape(len(cl), len(cr)) @ Ur).ravel())
        else:
            out.append(np.zeros(ml * mr))
    return np.concatenate(out)


def w_matrix(mps, dets, H, B, psi0):
    """W_ab = W(B_a, B_b) over the columns of B (module docstring)."""
    L = mps.L
    e0 = float(psi0 @ (H @ psi0))
    h0 = H @ psi0 - e0 * psi0
    lam_inv = [{c: np.linalg.inv(g) for c, g in gauge_matrix(mps, i).items()} for i in range(L - 1)]
    nb = B.shape[1]
    pieces = [site_pieces(mps, dets, B[:, a]) for a in range(nb)]
    # right-gauge pieces of every basis vector, flat per site: (nb, size_q)
    right_flat = [np.stack([firstorder.flat(mps, q, pieces[b][1][q]) for b in range(nb)]) for q in range(L)]
    half = np.zeros((nb, nb))  # half[a, b] = sum_{p<q} <Phi_pq[a, b] | h0>
    for a in range(nb):
        bl = pieces[a][0]
        # L1_p[a] = (Q^L G_p[a]) Lambda_p^{-1}
        l1 = []
        for p in range(L - 1):
            l1.append({(s, n): blk @ lam_inv[p][firstorder._right_sector(mps, p, s, n)]
                       for (s, n), blk in bl[p].items()})
        for q in range(1, L):
            gam = np.zeros(mps.site_size(q))
            for p in range(q):
                Lt = list(mps.Lt)
                Lt[p] = l1[p]
                gam += _project(mps, dets, Lt, q, h0)
            half[a] += right_flat[q] @ gam
    return half + half.T


def rpa_matrices(mps, dets, H, tol=1e-10):
    """(E0, A, W, B): the TDA matrix A = B^T (H - E0) B, the second-order
    matrix W, and the orthonormal tangent basis B with Psi0 removed."""
    psi0, B = response.tangent_space(mps, dets, tol)
    e0 = float(psi0 @ (H @ psi0))
    A = B.T @ (H @ B) - e0 * np.eye(B.shape[1])
    A = 0.5 * (A + A.T)
    return e0, A, w_matrix(mps, dets, H, B, psi0), B


def rpa_solve(A, W):
    """Positive eigenvalues of [[A, W], [-W, -A]] in ascending order (the
    RPA roots of eq. dmrgrpa in an orthonormal basis)."""
    n = A.shape[0]
    M = np.block([[A, W], [-W, -A]])
    w = np.linalg.eigvals(M)
    assert np.abs(w.imag).max() <= 1e-8 * max(1.0, np.abs(w.real).max()), "complex RPA roots (unstable reference)"
    w = np.sort(w.real)
    return w[n:]


def rpa_roots(mps, dets, H, nroots, tol=1e-10):
    """(E0, the nroots lowest RPA excitation energies, the nroots lowest TDA
    excitation energies) of the MPS reference."""
    e0, A, W, _ = rpa_matrices(mps, dets, H, tol)
    return e0, rpa_solve(A, W)[:nroots], np.linalg.eigvalsh(A)[:nroots]


def stationary_hamiltonian(mps, dets, H):
    """A symmetric matrix H' = H - t Psi0^T - Psi0 t^T, t the tangent-space
    component of (H - E0) Psi0, for which the reference is a stationary
    point of the energy on the MPS manifold (P_i^T (H' - E0) Psi0 = 0 at
    every site) with the same E0; used to build stationary references for
    checks that hold only there."""
    psi0 = mpsvec.mps_to_fci(mps, dets)
    psi0 = psi0 / np.linalg.norm(psi0)
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    e0 = float(psi0 @ Hd @ psi0)
    T, _ = tda.tangent_basis(mps, dets)
    t = T @ (T.T @ (Hd @ psi0 - e0 * psi0))
    return Hd - np.outer(t, psi0) - np.outer(psi0, t)
