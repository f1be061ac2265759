"""Brute-force Fock-space Hamiltonian for tiny systems (oracle; test only).

An independent construction used to pin fci.py: every ladder operator is an
explicit 2^(2L) x 2^(2L) Jordan-Wigner matrix (Kronecker products of 2x2
factors), and every term of H is formed as the literal product
a+_{ps} a+_{rt} a_{st} a_{qs}.  Basis index = bit string over modes with
mode 2i = (i, alpha), 2i+1 = (i, beta); the string of a mode's JW factor
runs over all lower modes.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def annihilator(nmodes, m):
    """Matrix of a_m on the full Fock space, basis index = bit string."""
    dim = 1 << nmodes
    rows, cols, vals = [], [], []
    for s in range(dim):
        if s >> m & 1:
            rows.append(s ^ (1 << m))
            cols.append(s)
            vals.append((-1) ** bin(s & ((1 << m) - 1)).count("1"))
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim))


def fock_hamiltonian(h, eri, ecore):
    L = h.shape[0]
    nm = 2 * L
    a = [annihilator(nm, m) for m in range(nm)]
    c = [x.T for x in a]
    dim = 1 << nm
    H = ecore * sp.identity(dim, format="csr")
    for p in range(L):
        for q in range(L):
            for s in range(2):
                H += h[p, q] * c[2 * p + s] @ a[2 * q + s]
    for p in range(L):
        for q in range(L):
            for r in range(L):
                for s_ in range(L):
                    v = eri[p, q, r, s_]
                    if v == 0.0:
                        continue
                    for sg in range(2):
                        for tg in range(2):
                            H += 0.5 * v * (c[2 * p + sg] @ c[2 * r + tg]
                                            @ a[2 * s_ + tg] @ a[2 * q + sg])
    return H.toarray()


def sector_indices(L, Na, Nb):
    out = []
    for s in range(1 << (2 * L)):
        na = sum(s >> (2 * i) & 1 for i in range(L))
        nb = sum(s >> (2 * i + 1) & 1 for i in range(L))
        if na == Na and nb == Nb:
            out.append(s)
    return np.array(out, dtype=np.int64)
