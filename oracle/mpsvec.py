"""MPS <-> FCI-vector maps and the dense explicit effective Hamiltonian
(oracle; test infrastructure only).

Definitions followed (Sec. II A of the paper): the renormalized left states
|l_{i-1}> are products of the left-orthonormal tensors L^{n_1}..L^{n_{i-1}},
the right states |r_i> products of R^{n_{i+1}}..R^{n_k}; the one-site product
basis |l n r> spans the site-i problem and the effective Hamiltonian is
H_i = <l' n' r'| H |l n r>, i.e. P_i^T H P_i with P_i the matrix whose columns
are those product states written as FCI vectors.  The two-site problem uses
|l n1 n2 r>.  Column order is the library's flat block order (blocks by
(left sector, n[, n2]), row-major inside a block).
"""
from __future__ import annotations

import numpy as np

QN = [(0, 0), (1, 0), (0, 1), (1, 1)]


def _left_states(mps, tensors, upto):
    """Left states of sites 0..upto-1: {sector a: (configs, matrix configs x m_a)}."""
    states = {0: (np.zeros(1, np.int64), np.ones((1, 1)))}
    for i in range(upto):
        idx = mps.sector_index(i + 1)
        new = {}
        for (a, n), blk in tensors[i].items():
            if a not in states:
                continue
            cfg, mat = states[a]
            q = mps.bonds[i][a][0]
            c = idx[(q[0] + QN[n][0], q[1] + QN[n][1])]
            new.setdefault(c, []).append((cfg | (np.int64(n) << (2 * i)), mat @ blk))
        states = {c: (np.concatenate([x[0] for x in v]), np.concatenate([x[1] for x in v]))
                  for c, v in new.items()}
    return states


def _right_states(mps, tensors, frm):
    """Right states of sites frm..L-1: {sector c at bond frm: (configs, configs x m_c)}."""
    L = mps.L
    states = {0: (np.zeros(1, np.int64), np.ones((1, 1)))}  # bond L, sector 0
    for i in range(L - 1, frm - 1, -1):
        idx = mps.sector_index(i + 1)
        new = {}
        for (a, n), blk in tensors[i].items():
            q = mps.bonds[i][a][0]
            c = idx[(q[0] + QN[n][0], q[1] + QN[n][1])]
            if c not in states:
                continue
            cfg, mat = states[c]
            # |r_a> = sum_n,c R[a, n, c] |n>|r_c>: configs x m_a matrix
            new.setdefault(a, []).append((cfg | (np.int64(n) << (2 * i)), mat @ blk.T))
        states = {a: (np.concatenate([x[0] for x in v]), np.concatenate([x[1] for x in v]))
                  for a, v in new.items()}
    return states


def mps_to_fci(mps, dets, tensors=None, site=None):
    """FCI vector of the MPS.  By default the left-canonical form
    L_0..L_{L-2} C_{L-1}; with site=i the mixed form L..L C_i R..R."""
    L = mps.L
    if site is None:
        site = L - 1
    left = _left_states(mps, mps.Lt, site)
    right = _right_states(mps, mps.Rt, site + 1)
    psi = np.zeros(len(dets))
    idx = mps.sector_index(site + 1)
    for (a, n), blk in mps.Ct[site].items():
        q = mps.bonds[site][a][0]
        c = idx[(q[0] + QN[n][0], q[1] + QN[n][1])]
        if a not in left or c not in right:
            continue
        cl, ml = left[a]
        cr, mr = right[c]
        amp = ml @ blk @ mr.T
        cfg = cl[:, None] | (np.int64(n) << (2 * site)) | cr[None, :]
        pos = np.searchsorted(dets, cfg.ravel())
        ok = (pos < len(dets)) & (dets[np.minimum(pos, len(dets) - 1)] == cfg.ravel())
        assert ok.all(), "configuration outside the determinant sector"
        np.add.at(psi, pos, amp.ravel())
    return psi


def site_basis(mps, dets, i):
    """P_i: FCI-space columns |l n r> for the one-site problem at site i."""
    left = _left_states(mps, mps.Lt, i)
    right = _right_states(mps, mps.Rt, i + 1)
    cols = []
    for a, n, c in mps.block_keys(i):
        ml_dim = mps.bonds[i][a][1]
        mr_dim = mps.bonds[i + 1][c][1]
        P = np.zeros((len(dets), ml_dim * mr_dim))
        if a in left and c in right:
            cl, ml = left[a]
            cr, mr = right[c]
            cfg = cl[:, None] | (np.int64(n) << (2 * i)) | cr[None, :]
            pos = np.searchsorted(dets, cfg.ravel())
            vals = np.einsum("xl,yr->xylr", ml, mr).reshape(len(cl) * len(cr), -1)
            P[pos] += vals
        cols.append(P)
    return np.concatenate(cols, axis=1) if cols else np.zeros((len(dets), 0))


def two_site_basis(mps, dets, i):
    """P_{i,i+1}: columns |l n1 n2 r> with l at bond i and r at bond i+2."""
    from synth import two_site_keys  # block order only (data format)
    left = _left_states(mps, mps.Lt, i)
    right = _right_states(mps, mps.Rt, i + 2)
    cols = []
    for a, n1, n2, c in two_site_keys(mps, i):
        ml_dim = mps.bonds[i][a][1]
        mr_dim = mps.bonds[i + 2][c][1]
        P = np.zeros((len(dets), ml_dim * mr_dim))
        if a in left and c in right:
            cl, ml = left[a]
            cr, mr = right[c]
            nb = (np.int64(n1) << (2 * i)) | (np.int64(n2) << (2 * i + 2))
            cfg = cl[:, None] | nb | cr[None, :]
            pos = np.searchsorted(dets, cfg.ravel())
            vals = np.einsum("xl,yr->xylr", ml, mr).reshape(len(cl) * len(cr), -1)
            P[pos] += vals
        cols.append(P)
    return np.concatenate(cols, axis=1) if cols else np.zeros((len(dets), 0))


def _product_blocks(mps, i, width):
    """(block keys, left states, right states, site shift) of the one- or
    two-site product basis at site i, in the flat column order."""
    from synth import two_site_keys  # block order only (data format)
    left = _left_states(mps, mps.Lt, i)
    right = _right_states(mps, mps.Rt, i + width)
    blocks = []
    if width == 1:
        for a, n, c in mps.block_keys(i):
            blocks.append((a, np.int64(n) << (2 * i), c, mps.bonds[i][a][1], mps.bonds[i + 1][c][1]))
    else:
        for a, n1, n2, c in two_site_keys(mps, i):
            nb = (np.int64(n1) << (2 * i)) | (np.int64(n2) << (2 * i + 2))
            blocks.append((a, nb, c, mps.bonds[i][a][1], mps.bonds[i + 2][c][1]))
    return blocks, left, right


def heff_apply(H, mps, dets, i, C, width=1):
    """sigma = P^T H P c for each row c of C, without forming P: P c is the
    FCI vector sum over blocks of |l> c_block <r| (the expansion of the
    product basis), H acts as a sparse matrix, and P^T v contracts v with
    the same left and right states block by block."""
    blocks, left, right = _product_blocks(mps, i, width)
    C = np.atleast_2d(C)
    out = np.zeros_like(C, dtype=np.float64)
    where = []
    off = 0
    for a, nb, c, ml, mr in blocks:
        if a in left and c in right:
            cl, Ul = left[a]
            cr, Ur = right[c]
            cfg = (cl[:, None] | nb | cr[None, :]).ravel()
            pos = np.searchsorted(dets, cfg)
            where.append((off, ml, mr, Ul, Ur, pos))
        off += ml * mr
    for v in range(C.shape[0]):
        psi = np.zeros(len(dets))
        for o, ml, mr, Ul, Ur, pos in where:
            blk = C[v, o:o + ml * mr].reshape(ml, mr)
            np.add.at(psi, pos, (Ul @ blk @ Ur.T).ravel())
        hpsi = H @ psi
        for o, ml, mr, Ul, Ur, pos in where:
            V = hpsi[pos].reshape(Ul.shape[0], Ur.shape[0])
            out[v, o:o + ml * mr] = (Ul.T @ V @ Ur).ravel()
    return out


def heff(H, P):
    """Dense explicit effective Hamiltonian P^T H P."""
    return P.T @ (H @ P)


def energy(H, psi):
    return float(psi @ (H @ psi) / (psi @ psi))


def fci_to_mps(psi, dets, L, Na, Nb, cut=1e-12):
    """Exact MPS of an FCI vector by successive SVDs (left-orthonormal sites,
    the norm in the last site); bond dims are the Schmidt ranks.  Returns
    (bonds, tensors) in the synth block format, used to build an exact
    reference state for the full-space checks."""
    # amplitudes keyed by configuration
    amp = dict(zip(dets.tolist(), psi.tolist()))
    # current "carry": for each left sector, list of (config prefix rows) x
    # remaining-config columns; do it by recursion on site.
    # Represent the state as a matrix rows = left basis states, cols = suffix configs.
    rows = {(0, 0): np.ones((1, 1))}
    suffix = {}
    for d, v in amp.items():
        suffix.setdefault((0, 0), {})[d] = v
    # suffix[q][config] -> amplitude vector over left states of sector q
    suffix = {(0, 0): {d: np.array([v]) for d, v in amp.items()}}
    bonds = [[((0, 0), 1)]]
    tensors = []
    for i in range(L):
        # group by new sector and by the suffix (sites > i)
        new = {}
        for q, tab in suffix.items():
            for d, vec in tab.items():
                n = (d >> (2 * i)) & 3
                qc = (q[0] + QN[n][0], q[1] + QN[n][1])
                rest = d & ~((np.int64(1) << (2 * i + 2)) - 1) if i < L - 1 else 0
                new.setdefault(qc, {}).setdefault(int(rest), {})[(q, n)] = vec
        # for each new sector build the matrix (left states x n) x suffixes
        bond_q = sorted(new.keys())
        prev_index = {q: k for k, (q, _) in enumerate(bonds[-1])}
        prev_dim = {q: d for q, d in bonds[-1]}
        T = {}
        newsuffix = {}
        newbond = []
        for qc in bond_q:
            tab = new[qc]
            rowkeys = sorted({k for col in tab.values() for k in col},
                             key=lambda x: (prev_index[x[0]], x[1]))
            offs, tot = {}, 0
            for k in rowkeys:
                offs[k] = tot
                tot += prev_dim[k[0]]
            sufs = sorted(tab.keys())
            Mat = np.zeros((tot, len(sufs)))
            for j, s in enumerate(sufs):
                for k, vec in tab[s].items():
                    Mat[offs[k]:offs[k] + len(vec), j] = vec
            if i == L - 1:
                U, s, Vh = Mat, None, None
                keep_dim = 1
                carry = None
            else:
                U, s, Vh = np.linalg.svd(Mat, full_matrices=False)
                keep = s > cut * s.max() if s.size else np.zeros(0, bool)
                U, s, Vh = U[:, keep], s[keep], Vh[keep]
                keep_dim = len(s)
                carry = s[:, None] * Vh
            if keep_dim == 0:
                continue
            newbond.append((qc, keep_dim))
            for k in rowkeys:
                T[(prev_index[k[0]], k[1], qc)] = U[offs[k]:offs[k] + prev_dim[k[0]]]
            if carry is not None:
                newsuffix[qc] = {s_: carry[:, j] for j, s_ in enumerate(sufs)}
        idx_new = {q: k for k, (q, _) in enumerate(newbond)}
        tensors.append({(a, n): blk for (a, n, qc), blk in T.items() if qc in idx_new})
        bonds.append(newbond)
        suffix = newsuffix
    return bonds, tensors
