"""Test helpers: marshal synth MPS objects to the library's flat format and
back (data layout only)."""
import numpy as np

import synth


def mps_arrays(mps):
    nsec, sec = synth.bond_table(mps)
    Ld = np.concatenate([mps.flat("L", i) for i in range(mps.L)])
    Rd = np.concatenate([mps.flat("R", i) for i in range(mps.L)])
    Cd = np.concatenate([mps.flat("C", i) for i in range(mps.L)])
    lam = np.concatenate([mps.lam[b][a] for b in range(mps.L + 1) for a in range(len(mps.bonds[b]))])
    return nsec, sec, Ld, Rd, Cd, lam


def mps_from_arrays(L, Na, Nb, nsec, sec, Ld, Rd, Cd, lam):
    bonds, k = [], 0
    for b in range(L + 1):
        bonds.append([((int(sec[k + s][0]), int(sec[k + s][1])), int(sec[k + s][2])) for s in range(nsec[b])])
        k += nsec[b]
    m = synth.MPS(L, Na, Nb, bonds)
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


def make_context(prob_h, prob_eri, L, Na, Nb, ecore=0.0, device=0):
    import paper_1311_1646_amd as lib
    return lib.Context(L, Na, Nb, prob_h, prob_eri, ecore, device=device)
