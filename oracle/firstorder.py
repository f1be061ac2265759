"""First-order MPS wavefunctions and the DMRG-TDA sigma vector (oracle; test
infrastructure only).

Definitions followed:
  * Sec. II B, eq. psi1st: the first-order change of an MPS is the sum over
    sites of the wavefunction with one site tensor replaced by its first-order
    tensor.  In the mixed gauge centred at site i (Sec. II B, the
    gauge-transformed forms behind eqs. gauge_bwd / gauge_fwd, and Sec. III D)
    it reads
        Psi1 = sum_{j<i} L..L L1_j L..L C_i R..R          (centre tensor C_i)
             + L..L C1_i R..R
             + sum_{j>i} L..L C_i R..R R1_j R..R
  * Sec. II B, eqs. left-orthoSeb / right-orthoSeb: the first-order tensors
    satisfy L_j^T L1_j = 0 and R1_j R_j^T = 0 (contracted over the left
    index and the site index, resp. the site index and the right index).
    Arbitrary tensors are brought there by the projectors
    Q^L X = X - L (L^T X) and X Q^R = X - (X R^T) R.
  * Sec. III D, eq. sigv1 (with eq. sigv2): the TDA sigma at site i is the
    projection of H Psi1 onto the one-site product basis of site i,
    sigma_i = P_i^T H Psi1.  Its first-order left part (first line of eq.
    sigv2) is P_i^T H (sum_{j<i} L..L1_j..L C R..R) for a given centre C.

Tensors are dicts {(a, n): block} as in synth.MPS; flat vectors use the
library's block order (synth.MPS.block_keys).
"""
from __future__ import annotations

import numpy as np

from . import mpsvec

QN = [(0, 0), (1, 0), (0, 1), (1, 1)]


def blocks(mps, i, x):
    """Flat one-site vector at site i -> dict {(a, n): block}."""
    out, off = {}, 0
    for a, n, c in mps.block_keys(i):
        r, cc = mps.bonds[i][a][1], mps.bonds[i + 1][c][1]
        out[(a, n)] = np.asarray(x[off:off + r * cc], dtype=np.float64).reshape(r, cc)
        off += r * cc
    assert off == len(x), "vector length differs from the site's layout"
    return out


def flat(mps, i, T):
    """dict {(a, n): block} -> flat one-site vector at site i."""
    return np.concatenate([T[(a, n)].ravel() for a, n, _ in mps.block_keys(i)])


def _right_sector(mps, i, a, n):
    q = mps.bonds[i][a][0]
    return mps.sector_index(i + 1)[(q[0] + QN[n][0], q[1] + QN[n][1])]


def q_left(mps, i, X):
    """Q^L X = X - L_i (L_i^T X): for each right sector c, the rows (a, n)
    feeding c form one matrix; L^T X contracts those rows (left-orthoSeb)."""
    L = mps.Lt[i]
    G = {}
    for (a, n), x in X.items():
        c = _right_sector(mps, i, a, n)
        g = L[(a, n)].T @ x
        G[c] = G[c] + g if c in G else g
    return {(a, n): x - L[(a, n)] @ G[_right_sector(mps, i, a, n)] for (a, n), x in X.items()}


def q_right(mps, i, X):
    """X Q^R = X - (X R_i^T) R_i: for each left sector a, the columns (n, c)
    of a form one matrix; X R^T contracts them (right-orthoSeb)."""
    R = mps.Rt[i]
    G = {}
    for (a, n), x in X.items():
        g = x @ R[(a, n)].T
        G[a] = G[a] + g if a in G else g
    return {(a, n): x - G[a] @ R[(a, n)] for (a, n), x in X.items()}


def fci_vector(mps, dets, Lt, centre, Rt, site):
    """FCI vector of L..L (tensors Lt[0..site-1]) centre R..R (Rt[site+1..])."""
    left = mpsvec._left_states(mps, Lt, site)
    right = mpsvec._right_states(mps, Rt, site + 1)
    psi = np.zeros(len(dets))
    for (a, n), blk in centre.items():
        c = _right_sector(mps, site, a, n)
        if a not in left or c not in right:
            continue
        cl, ml = left[a]
        cr, mr = right[c]
        cfg = (cl[:, None] | (np.int64(n) << (2 * site)) | cr[None, :]).ravel()
        pos = np.searchsorted(dets, cfg)
        assert (dets[np.minimum(pos, len(dets) - 1)] == cfg).all(), "configuration outside the sector"
        np.add.at(psi, pos, (ml @ blk @ mr.T).ravel())
    return psi


def first_order_psi(mps, dets, i, L1, C1, R1, centre=None):
    """Psi1 in the mixed gauge at site i (module docstring).  L1: {j: tensor}
    for j < i, R1: {j: tensor} for j > i (dicts of blocks, projected here by
    Q^L / Q^R); C1: centre tensor at i or None; centre: the zeroth-order
    centre of the L1 / R1 terms (default C_i of the MPS)."""
    C0 = mps.Ct[i] if centre is None else centre
    psi = np.zeros(len(dets))
    for j, X in L1.items():
        assert j < i
        Lt = list(mps.Lt)
        Lt[j] = q_left(mps, j, X)
        psi += fci_vector(mps, dets, Lt, C0, mps.Rt, i)
    if C1 is not None:
        psi += fci_vector(mps, dets, mps.Lt, C1, mps.Rt, i)
    for j, X in R1.items():
        assert j > i
        Rt = list(mps.Rt)
        Rt[j] = q_right(mps, j, X)
        psi += fci_vector(mps, dets, mps.Lt, C0, Rt, i)
    return psi


def site_project(mps, dets, i, v):
    """P_i^T v: the components of an FCI vector along the one-site product
    basis |l n r> of site i, block by block (no P formed)."""
    blocks_, left, right = mpsvec._product_blocks(mps, i, 1)
    out = []
    for a, nb, c, ml, mr in blocks_:
        if a in left and c in right:
            cl, Ul = left[a]
            cr, Ur = right[c]
            pos = np.searchsorted(dets, (cl[:, None] | nb | cr[None, :]).ravel())
            out.append((Ul.T @ v[pos].reshape(len(cl), len(cr)) @ Ur).ravel())
        else:
            out.append(np.zeros(ml * mr))
    return np.concatenate(out)


def tda_sigma(H, mps, dets, i, L1, C1, R1):
    """TDA sigma of eq. sigv1 at site i: P_i^T H Psi1."""
    return site_project(mps, dets, i, H @ first_order_psi(mps, dets, i, L1, C1, R1))


def dh_left(H, mps, dets, i, L1, C):
    """First line of eq. sigv2 applied to the centre C at site i:
    P_i^T H (sum_{j<i} L..L1_j..L C R..R)."""
    return site_project(mps, dets, i, H @ first_order_psi(mps, dets, i, L1, None, {}, centre=C))
