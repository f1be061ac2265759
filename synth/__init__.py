"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input generation only: integrals shaped like the paper's
workloads and random matrix product states in mixed-canonical form.  It
contains none of the method's arithmetic (no Hamiltonian application, no
renormalization, no sigma, no Davidson); both the CPU oracle and the GPU
library receive the same arrays from here.

Conventions (shared data format, not method):
  * sites are spatial orbitals; the local basis of a site is
    n = 0:|0>, 1:|alpha>, 2:|beta>, 3:|alpha beta> (= a+_alpha a+_beta |0>);
  * a bond b (0..L) sits left of site b and is labelled by the
    (n_alpha, n_beta) counted over sites 0..b-1 ("left counts");
  * a site tensor A_i has one dense block per (left sector a, n) whose right
    sector c = q_a + q(n) exists at bond i+1; block shape (dim_a, dim_c),
    row-major; blocks are ordered by a, then n.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

HARTREE_PER_EV = 1.0 / 27.211386245988
QN = [(0, 0), (1, 0), (0, 1), (1, 1)]  # (n_alpha, n_beta) of local states


# --------------------------------------------------------------------------
# Integrals
# --------------------------------------------------------------------------

def _sym_normal(rng, n, sigma):
    a = rng.normal(0.0, sigma, size=(n, n))
    return np.triu(a) + np.triu(a, 1).T


def random_integrals(L, seed, K, diag_lo, diag_hi, h_sigma=0.5, chol_sigma=0.1,
                     diag=None, chol_scale_block=None):
    """Random dense integrals: h symmetric N(0,h_sigma) plus an ascending
    diagonal shift; (pq|rs) = sum_K Lk_pq Lk_rs with Lk symmetric N(0,chol_sigma),
    which has the 8-fold symmetry of real orbitals and is positive semidefinite
    as a pair-space matrix."""
    rng = np.random.default_rng(seed)
    h = _sym_normal(rng, L, h_sigma)
    if diag is None:
        diag = np.linspace(diag_lo, diag_hi, L)
    h = h + np.diag(diag)
    chol = np.stack([_sym_normal(rng, L, chol_sigma) for _ in range(K)])
    if chol_scale_block is not None:
        blk, fac = chol_scale_block
        m = np.zeros((L, L), bool)
        m[np.ix_(blk, blk)] = True
        chol[:, m] *= fac
    eri = np.einsum("kpq,krs->pqrs", chol, chol)
    return h, eri, 0.0


def ppp_integrals(L, t0=-2.4, dt=0.1, U=11.13, a0=1.4, spacing=1.4):
    """Pariser-Parr-Pople chain in Hartree: alternating hopping
    t_i = t0 + dt*(-1)^i on bond (i,i+1), Ohno-decayed Coulomb
    V_ij = U/sqrt(1+(r_ij/a0)^2), (ii|jj) = V_ij, and h_ii = -sum_{j!=i} V_ij
    (the (n_i-1)(n_j-1) form; its constant is dropped, E_core = 0)."""
    h = np.zeros((L, L))
    for i in range(L - 1):
        t = t0 + dt * (-1) ** i
        h[i, i + 1] = h[i + 1, i] = t
    r = spacing * np.abs(np.subtract.outer(np.arange(L), np.arange(L)))
    V = U / np.sqrt(1.0 + (r / a0) ** 2)
    for i in range(L):
        h[i, i] = -(V[i].sum() - V[i, i])
    eri = np.zeros((L, L, L, L))
    for i in range(L):
        for j in range(L):
            eri[i, i, j, j] = V[i, j]
    return h * HARTREE_PER_EV, eri * HARTREE_PER_EV, 0.0


@dataclass
class Problem:
    name: str
    L: int
    Na: int
    Nb: int
    h: np.ndarray
    eri: np.ndarray
    ecore: float
    M: int
    nroots: int


def config(cfg: int, instance: int = 0, M: int | None = None) -> Problem:
    """Synthetic workloads standing in for the paper's molecules (whose
    integrals are not available): 0 small dense check, 1 PPP polyene chain,
    2 water-shaped dense, 3 batched instances, 4 [2Fe-2S]-shaped
    near-degenerate block."""
    seed = 1000 * cfg + instance
    if cfg == 0:
        L, N = 8, 8
        h, eri, e0 = random_integrals(L, seed, K=16, diag_lo=-2.0, diag_hi=0.0)
        P = Problem("rand-L8-N8", L, N // 2, N // 2, h, eri, e0, M or 64, 4)
    elif cfg == 1:
        L, N = 24, 24
        h, eri, e0 = ppp_integrals(L)
        P = Problem("ppp-L24-N24", L, N // 2, N // 2, h, eri, e0, M or 256, 6)
    elif cfg == 2:
        L, N = 24, 10
        h, eri, e0 = random_integrals(L, seed, K=72, diag_lo=-20.0, diag_hi=2.0)
        P = Problem("rand-L24-N10", L, N // 2, N // 2, h, eri, e0, M or 500, 8)
    elif cfg == 3:
        rng = np.random.default_rng(seed)
        L = int(rng.integers(8, 17))
        Mi = int(rng.integers(32, 257))
        h, eri, e0 = random_integrals(L, seed, K=16, diag_lo=-2.0, diag_hi=0.0)
        P = Problem(f"batch-L{L}", L, L // 2, L - L // 2, h, eri, e0, M or Mi, 4)
    elif cfg == 4:
        L, N = 36, 30
        blk = list(range(10, 20))
        others = [i for i in range(L) if i not in blk]
        diag = np.zeros(L)
        diag[others] = np.linspace(-2.0, 0.0, len(others))
        diag[blk] = np.linspace(-0.2, 0.2, len(blk))
        h, eri, e0 = random_integrals(L, seed, K=108, diag_lo=0, diag_hi=0,
                                      diag=diag, chol_scale_block=(blk, 3.0))
        P = Problem("fe2s2-L36-N30", L, N // 2, N // 2, h, eri, e0, M or 1000, 16)
    else:
        raise ValueError(cfg)
    return P


# --------------------------------------------------------------------------
# Bond sector tables and random mixed-canonical MPS
# --------------------------------------------------------------------------

def full_sector_dims(L, Na, Nb, b):
    """Exact (left-count) sectors at bond b with min(left, right) Fock dims."""
    out = []
    for na in range(0, min(b, Na) + 1):
        if Na - na > L - b:
            continue
        for nb in range(0, min(b, Nb) + 1):
            if Nb - nb > L - b:
                continue
            dl = math.comb(b, na) * math.comb(b, nb)
            dr = math.comb(L - b, Na - na) * math.comb(L - b, Nb - nb)
            out.append(((na, nb), min(dl, dr)))
    return out


def truncated_bond_dims(L, Na, Nb, M, width=1.1):
    """Distribute M states over each bond's sectors with Gaussian weights
    around the mean filling, capped by the exact dims (bond 0 and L have dim 1)."""
    bonds = []
    for b in range(L + 1):
        full = full_sector_dims(L, Na, Nb, b)
        tot = sum(d for _, d in full)
        if tot <= M:
            bonds.append([(q, d) for q, d in full])
            continue
        ca, cb = Na * b / L, Nb * b / L
        w = np.array([math.exp(-((q[0] - ca) ** 2 + (q[1] - cb) ** 2) / (2 * width ** 2))
                      for q, _ in full])
        cap = np.array([d for _, d in full], float)
        alloc = np.zeros(len(full))
        remaining = float(M)
        active = np.ones(len(full), bool)
        for _ in range(64):  # water-filling with caps
            if remaining <= 0.5 or not active.any():
                break
            share = remaining * w * active / (w * active).sum()
            new = np.minimum(alloc + share, cap)
            remaining -= (new - alloc).sum()
            alloc = new
            active = alloc < cap - 1e-9
        dims = np.floor(alloc).astype(int)
        short = M - dims.sum()
        order = np.argsort(-(alloc - dims))
        for k in order:
            if short <= 0:
                break
            if dims[k] < cap[k]:
                dims[k] += 1
                short -= 1
        bonds.append([(q, int(d)) for (q, _), d in zip(full, dims) if d > 0])
    return bonds


@dataclass
class MPS:
    """Mixed-canonical MPS: for every site i the left-orthonormal L[i], the
    right-orthonormal R[i] and C[i] = L[i] Lam[i+1] = Lam[i] R[i]; Lam[b] is the
    (diagonal, per sector) Schmidt spectrum at bond b.  Tensors are dicts
    {(a, n): block}, bonds are lists of ((na, nb), dim)."""
    L: int
    Na: int
    Nb: int
    bonds: list
    Lt: list = field(default_factory=list)
    Rt: list = field(default_factory=list)
    Ct: list = field(default_factory=list)
    lam: list = field(default_factory=list)  # lam[b] = {a: vector}

    def sector_index(self, b):
        return {q: k for k, (q, _) in enumerate(self.bonds[b])}

    def block_keys(self, i):
        """Canonical block order of a site-i tensor: (a, n, c)."""
        left = self.bonds[i]
        right = self.sector_index(i + 1)
        keys = []
        for a, (q, _) in enumerate(left):
            for n in range(4):
                qc = (q[0] + QN[n][0], q[1] + QN[n][1])
                if qc in right:
                    keys.append((a, n, right[qc]))
        return keys

    def flat(self, which, i):
        T = {"L": self.Lt, "R": self.Rt, "C": self.Ct}[which][i]
        return np.concatenate([T[(a, n)].ravel() for a, n, _ in self.block_keys(i)]) \
            if self.block_keys(i) else np.zeros(0)

    def site_size(self, i):
        return sum(self.bonds[i][a][1] * self.bonds[i + 1][c][1] for a, n, c in self.block_keys(i))


def _left_groups(mps, i, dims_l, dims_r):
    """For site i: map right sector c -> list of (a, n) rows feeding it."""
    left = mps.bonds[i]
    right = mps.sector_index(i + 1)
    g = {}
    for a, (q, _) in enumerate(left):
        for n in range(4):
            qc = (q[0] + QN[n][0], q[1] + QN[n][1])
            if qc in right:
                g.setdefault(right[qc], []).append((a, n))
    return g


def _right_groups(mps, i):
    """For site i: map left sector a -> list of (n, c) columns."""
    right = mps.sector_index(i + 1)
    g = {}
    for a, (q, _) in enumerate(mps.bonds[i]):
        for n in range(4):
            qc = (q[0] + QN[n][0], q[1] + QN[n][1])
            if qc in right:
                g.setdefault(a, []).append((n, right[qc]))
    return g


def _split_cols(mat, widths):
    out, off = [], 0
    for w in widths:
        out.append(mat[:, off:off + w])
        off += w
    return out


def _lr_pass(mps, A, cut):
    """Left-to-right SVD pass: A[i] left-orthonormal for i < L-1, zero
    singular values dropped (bond dims shrink), the rest carried right."""
    L = mps.L
    changed = False
    for i in range(L - 1):
        groups = _left_groups(mps, i, None, None)
        newL, carry, newdims = {}, {}, {}
        for c, rows in groups.items():
            mat = np.concatenate([A[i][(a, n)] for a, n in rows], axis=0)
            U, s, Vh = np.linalg.svd(mat, full_matrices=False)
            keep = s > cut * max(s.max(), 1e-300)
            U, s, Vh = U[:, keep], s[keep], Vh[keep]
            off = 0
            for a, n in rows:
                h_ = A[i][(a, n)].shape[0]
                newL[(a, n)] = U[off:off + h_]
                off += h_
            carry[c] = s[:, None] * Vh
            newdims[c] = len(s)
        for (a2, n2), blk in list(A[i + 1].items()):
            A[i + 1][(a2, n2)] = carry[a2] @ blk
        old = mps.bonds[i + 1]
        mps.bonds[i + 1] = [(q, newdims[k]) for k, (q, _) in enumerate(old)]
        changed |= any(d0 != d1 for (_, d0), (_, d1) in zip(old, mps.bonds[i + 1]))
        A[i] = newL
    return changed


def _rl_pass(mps, A, cut):
    """Right-to-left SVD pass: A[i] right-orthonormal for i > 0."""
    L = mps.L
    changed = False
    for i in range(L - 1, 0, -1):
        groups = _right_groups(mps, i)
        newR, carry, newdims = {}, {}, {}
        for a, cols in groups.items():
            mat = np.concatenate([A[i][(a, n)] for n, c in cols], axis=1)
            U, s, Vh = np.linalg.svd(mat, full_matrices=False)
            keep = s > cut * max(s.max(), 1e-300)
            U, s, Vh = U[:, keep], s[keep], Vh[keep]
            for (n, c), blk in zip(cols, _split_cols(Vh, [A[i][(a, n)].shape[1] for n, c in cols])):
                newR[(a, n)] = blk
            carry[a] = U * s
            newdims[a] = len(s)
        for (a2, n2), blk in list(A[i - 1].items()):
            qa = mps.bonds[i - 1][a2][0]
            qc = (qa[0] + QN[n2][0], qa[1] + QN[n2][1])
            A[i - 1][(a2, n2)] = blk @ carry[mps.sector_index(i)[qc]]
        old = mps.bonds[i]
        mps.bonds[i] = [(q, newdims[k]) for k, (q, _) in enumerate(old)]
        changed |= any(d0 != d1 for (_, d0), (_, d1) in zip(old, mps.bonds[i]))
        A[i] = newR
    return changed


def _prune_empty(mps, A):
    """Remove sectors whose dimension dropped to zero (and their blocks)."""
    for b in range(mps.L + 1):
        if all(d > 0 for _, d in mps.bonds[b]):
            continue
        keep = [k for k, (_, d) in enumerate(mps.bonds[b]) if d > 0]
        remap = {old: new for new, old in enumerate(keep)}
        alive = {mps.bonds[b][k][0] for k in keep}
        if b < mps.L:  # left index of site b
            A[b] = {(remap[a], n): v for (a, n), v in A[b].items() if a in remap}
        if b > 0:      # right index of site b-1
            def _ok(a, n):
                q = mps.bonds[b - 1][a][0]
                return (q[0] + QN[n][0], q[1] + QN[n][1]) in alive
            A[b - 1] = {k: v for k, v in A[b - 1].items() if _ok(*k)}
        mps.bonds[b] = [mps.bonds[b][k] for k in keep]


def random_mps(L, Na, Nb, M, seed, width=1.1, cut=1e-10):
    """Random normalized U(1)xU(1) MPS brought to mixed-canonical form with
    diagonal (Schmidt) Lambda at every bond.  Directions with singular values
    below cut * max are removed first, so every Lambda is invertible and the
    bond dims are minimal."""
    rng = np.random.default_rng(seed)
    bonds = truncated_bond_dims(L, Na, Nb, M, width)
    mps = MPS(L, Na, Nb, [list(b) for b in bonds])
    A = []
    for i in range(L):
        T = {}
        for a, n, c in mps.block_keys(i):
            T[(a, n)] = rng.normal(size=(mps.bonds[i][a][1], mps.bonds[i + 1][c][1]))
        A.append(T)
    return canonical_from_tensors(L, Na, Nb, mps.bonds, A, cut)


def canonical_from_tensors(L, Na, Nb, bonds, A, cut=1e-10):
    """Mixed-canonical form (L_i, R_i, C_i, diagonal Lambda) of the MPS with
    site tensors A (synth block format); the state is normalized."""
    mps = MPS(L, Na, Nb, [list(b) for b in bonds])
    A = [dict(t) for t in A]
    for _ in range(8):
        ch1 = _lr_pass(mps, A, cut)
        _prune_empty(mps, A)
        ch2 = _rl_pass(mps, A, cut)
        _prune_empty(mps, A)
        if not (ch1 or ch2):
            break
    nrm = math.sqrt(sum(float((b ** 2).sum()) for b in A[0].values()))
    for k in A[0]:
        A[0][k] /= nrm
    Rt = [dict(t) for t in A]
    Lt, Ct, lam = [None] * L, [None] * L, [None] * (L + 1)
    lam[0] = {0: np.ones(1)}
    C = {k: v.copy() for k, v in A[0].items()}
    for i in range(L):
        if i == L - 1:
            Lt[i] = {k: v.copy() for k, v in C.items()}
            Ct[i] = {k: v.copy() for k, v in C.items()}
            lam[L] = {0: np.ones(1)}
            break
        groups = _left_groups(mps, i, None, None)
        Li, Ci, lam_i, V = {}, {}, {}, {}
        for c, rows in groups.items():
            mat = np.concatenate([C[(a, n)] for a, n in rows], axis=0)
            U, s, Vh = np.linalg.svd(mat, full_matrices=False)
            if len(s) != mat.shape[1] or s.min() <= cut * s.max():
                raise RuntimeError("rank-deficient bond in canonical pass")
            off = 0
            for a, n in rows:
                h_ = C[(a, n)].shape[0]
                Li[(a, n)] = U[off:off + h_]
                Ci[(a, n)] = U[off:off + h_] * s
                off += h_
            lam_i[c] = s
            V[c] = Vh
        Lt[i], Ct[i], lam[i + 1] = Li, Ci, lam_i
        idx1 = mps.sector_index(i + 1)
        for (a, n), blk in Rt[i].items():   # columns of R[i] into the new basis
            qa = mps.bonds[i][a][0]
            c = idx1[(qa[0] + QN[n][0], qa[1] + QN[n][1])]
            Rt[i][(a, n)] = blk @ V[c].T
        Rn, Cn = {}, {}
        for (a, n), blk in Rt[i + 1].items():
            Rn[(a, n)] = V[a] @ blk
            Cn[(a, n)] = lam_i[a][:, None] * Rn[(a, n)]
        Rt[i + 1] = Rn
        C = Cn
    mps.Lt, mps.Rt, mps.Ct, mps.lam = Lt, Rt, Ct, lam
    return mps


def random_site_vectors(mps, i, nvec, seed):
    """Random coefficient tensors in the site-i block layout (flat, fp64)."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=(nvec, mps.site_size(i)))


def two_site_keys(mps, i):
    """Canonical block order of a two-site (i, i+1) coefficient tensor:
    (a, n1, n2, c) with a at bond i and c at bond i+2."""
    right = mps.sector_index(i + 2)
    keys = []
    for a, (q, _) in enumerate(mps.bonds[i]):
        for n1 in range(4):
            for n2 in range(4):
                qc = (q[0] + QN[n1][0] + QN[n2][0], q[1] + QN[n1][1] + QN[n2][1])
                if qc in right:
                    keys.append((a, n1, n2, right[qc]))
    return keys


def bond_table(mps):
    """Flat int32 description of all bonds: for each bond b the count of
    sectors, then (na, nb, dim) per sector."""
    counts = np.array([len(b) for b in mps.bonds], np.int32)
    secs = np.array([[q[0], q[1], d] for b in mps.bonds for q, d in b], np.int32).ravel()
    return counts, secs


# --------------------------------------------------------------------------
# Flat arrays of the library's MPS import / export format (data layout only)
# --------------------------------------------------------------------------

def mps_arrays(mps):
    """(nsec, sectors, L data, R data, C data, lam) of an MPS in the flat
    format of dmrg_import_mps."""
    nsec, sec = bond_table(mps)
    Ld = np.concatenate([mps.flat("L", i) for i in range(mps.L)])
    Rd = np.concatenate([mps.flat("R", i) for i in range(mps.L)])
    Cd = np.concatenate([mps.flat("C", i) for i in range(mps.L)])
    lam = np.concatenate([mps.lam[b][a] for b in range(mps.L + 1) for a in range(len(mps.bonds[b]))])
    return nsec, sec, Ld, Rd, Cd, lam


def mps_from_arrays(L, Na, Nb, nsec, sec, Ld, Rd, Cd, lam):
    """Inverse of mps_arrays (the arrays of dmrg_export_mps -> MPS)."""
    bonds, k = [], 0
    for b in range(L + 1):
        bonds.append([((int(sec[k + s][0]), int(sec[k + s][1])), int(sec[k + s][2])) for s in range(nsec[b])])
        k += nsec[b]
    m = MPS(L, Na, Nb, bonds)
    off = 0
    m.Lt, m.Rt, m.Ct = [], [], []
    for i in range(L):
        T = {"L": {}, "R": {}, "C": {}}
        for a, n, c in m.block_keys(i):
            r, cc = bonds[i][a][1], bonds[i + 1][c][1]
            for key, src in (("L", Ld), ("R", Rd), ("C", Cd)):
                T[key][(a, n)] = src[off:off + r * cc].reshape(r, cc).copy()
            off += r * cc
        m.Lt.append(T["L"])
        m.Rt.append(T["R"])
        m.Ct.append(T["C"])
    lo = 0
    m.lam = []
    for b in range(L + 1):
        d = {}
        for a, (_, dim) in enumerate(bonds[b]):
            d[a] = lam[lo:lo + dim].copy()
            lo += dim
        m.lam.append(d)
    return m
