"""Determinant-basis Hamiltonian and FCI (oracle; test infrastructure only).

H = E_core + sum_{pq,s} h_pq a+_{ps} a_{qs}
          + 1/2 sum_{pqrs, s t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}
for real orbitals, built in the determinant basis of fixed (N_alpha, N_beta)
from spin-summed excitation operators E_pq = sum_s a+_{ps} a_{qs} using
a+_p a+_r a_s a_q summed over spins = E_pq E_rs - delta_qr E_ps.

Determinants are bit strings over 2L spin-orbitals, mode 2i = (i, alpha),
2i+1 = (i, beta); a determinant is the product of creators of its occupied
modes in increasing mode order acting on the vacuum.  This is the same
ordering as the product basis |n_0 n_1 ...> of the MPS, so no extra sign
connects the two.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp


def determinants(L, Na, Nb):
    """Sorted bit strings of all determinants with Na alpha and Nb beta electrons."""
    dets = []
    for oa in itertools.combinations(range(L), Na):
        for ob in itertools.combinations(range(L), Nb):
            d = 0
            for i in oa:
                d |= 1 << (2 * i)
            for i in ob:
                d |= 1 << (2 * i + 1)
            dets.append(d)
    return np.array(sorted(dets), dtype=np.int64)


def _popcount(x):
    x = x.copy()
    c = np.zeros_like(x)
    while np.any(x):
        c += x & 1
        x >>= 1
    return c


def excitation(dets, p, q):
    """Sparse matrix of a+_p a_q (spin-orbitals) on the determinant list."""
    n = len(dets)
    bq, bp = np.int64(1) << q, np.int64(1) << p
    occ_q = (dets & bq) != 0
    d1 = dets ^ bq
    ok = occ_q & ((p == q) | ((d1 & bp) == 0))
    src = np.nonzero(ok)[0]
    if len(src) == 0:
        return sp.csr_matrix((n, n))
    d = dets[src]
    s1 = _popcount(d & (bq - 1))
    d1 = d ^ bq
    s2 = _popcount(d1 & (bp - 1))
    new = d1 | bp
    dst = np.searchsorted(dets, new)
    sign = np.where((s1 + s2) % 2 == 0, 1.0, -1.0)
    return sp.csr_matrix((sign, (dst, src)), shape=(n, n))


def hamiltonian(h, eri, ecore, Na, Nb):
    """Sparse FCI Hamiltonian in the (Na, Nb) determinant basis."""
    L = h.shape[0]
    dets = determinants(L, Na, Nb)
    n = len(dets)
    E = {}
    for p in range(L):
        for q in range(L):
            E[p, q] = excitation(dets, 2 * p, 2 * q) + excitation(dets, 2 * p + 1, 2 * q + 1)
    H = sp.identity(n, format="csr") * ecore
    for p in range(L):
        for q in range(L):
            if h[p, q] != 0.0:
                H = H + h[p, q] * E[p, q]
    # two-body: 1/2 sum (pq|rs) (E_pq E_rs - delta_qr E_ps)
    for p in range(L):
        for q in range(L):
            G = sp.csr_matrix((n, n))
            for r in range(L):
                for s in range(L):
                    v = eri[p, q, r, s]
                    if v != 0.0:
                        G = G + v * E[r, s]
            H = H + 0.5 * (E[p, q] @ G)
    for p in range(L):
        for s in range(L):
            v = sum(eri[p, q, q, s] for q in range(L))
            if v != 0.0:
                H = H - 0.5 * v * E[p, s]
    return dets, H.tocsr()


DENSE_MAX = 6000


def fci(h, eri, ecore, Na, Nb, nroots=1):
    """Lowest eigenpairs of the FCI Hamiltonian by dense diagonalization
    (exact to rounding).  Larger spaces are refused: no test needs them, and
    an iterative eigensolver would be a second, unpinned code path."""
    dets, H = hamiltonian(h, eri, ecore, Na, Nb)
    n = len(dets)
    if n > DENSE_MAX:
        raise ValueError(f"{n} determinants: the oracle diagonalizes at most {DENSE_MAX} densely")
    w, v = np.linalg.eigh(H.toarray())
    return dets, H, w[:nroots], v[:, :nroots]


def ndeterminants(L, Na, Nb):
    return math.comb(L, Na) * math.comb(L, Nb)
