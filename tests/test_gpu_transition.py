"""GPU transition densities of the DMRG-TDA roots (dmrg_tda_transition;
Sec. VI A) against the oracle's, root by root up to the arbitrary sign of
each root, and their square norms sum_pq gamma_pq^2 (the paper's
single-excitation diagnostic)."""
import numpy as np
import pytest

import synth
from oracle import fci, transition
from synth import mps_arrays, mps_from_arrays

pytestmark = pytest.mark.gpu


def _align(g, ref):
    s = np.sign(np.sum(g * ref, axis=(1, 2)))
    return g * s[:, None, None]


def _bound(r2, ev, e_all=None):
    # eigenvector error is first order in the residual: |d y| <~ |r| / gap,
    # and gamma is linear in y (|V Psi0| ~ 1 for a unit E_pq)
    gap = np.min(np.diff(ev)) if len(ev) > 1 else 1.0
    return 20.0 * np.sqrt(np.max(r2)) / gap + 1e-9


@pytest.mark.parametrize("L,Na,Nb,M,seed,n", [(4, 2, 2, 6, 3, 2), (6, 3, 3, 12, 11, 3)])
def test_transition_densities_match_oracle(L, Na, Nb, M, seed, n):
    import paper_1311_1646_amd as lib
    h, eri, _ = synth.random_integrals(L, seed=seed, K=6, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, M, seed=seed + 1)
    ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
    ctx.import_mps(*mps_arrays(mps))
    ctx.build_ops()
    om, et, r2, it, conv, g = ctx.tda_transition(n, max_iter=80, tol=1e-12, seed=3)
    dets, H = fci.hamiltonian(h, eri, 0.0, Na, Nb)
    e0, ev, ref = transition.tda_transition(mps, dets, H, Na, Nb, n)
    assert conv
    np.testing.assert_allclose(et, ev, atol=1e-8)
    assert np.min(np.diff(ev)) > 1e-4  # distinct roots: vectors unique up to sign
    err = np.abs(_align(g, ref) - ref).max()
    b = _bound(r2, ev)
    print(f"L={L}: |d gamma| {err:.2e} (bound {b:.1e}), square norms {np.round(np.sum(g ** 2, axis=(1, 2)), 6)}")
    assert err < b
    np.testing.assert_allclose(np.sum(g ** 2, axis=(1, 2)), np.sum(ref ** 2, axis=(1, 2)), atol=4 * b)


def test_ground_state_transition_densities():
    # config 0 (L=8) ground state at M=24: the DMRG-TDA roots and their
    # transition densities against the oracle on the exported MPS
    import paper_1311_1646_amd as lib
    p = synth.config(0)
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    ctx.sweep_ground([16, 24, 24, 24], davidson_tol=1e-12, davidson_max_iter=60, seed=2)
    mps = mps_from_arrays(p.L, p.Na, p.Nb, *ctx.export_mps())
    om, et, r2, it, conv, g = ctx.tda_transition(3, max_iter=120, max_space=24, tol=1e-12, seed=3)
    dets, H = fci.hamiltonian(p.h, p.eri, p.ecore, p.Na, p.Nb)
    e0, ev, ref = transition.tda_transition(mps, dets, H, p.Na, p.Nb, 3)
    assert conv
    np.testing.assert_allclose(et, ev, atol=1e-8)
    gaps = np.min(np.diff(ev))
    sq, sq_ref = np.sum(g ** 2, axis=(1, 2)), np.sum(ref ** 2, axis=(1, 2))
    print(f"config 0: square norms {np.round(sq, 6)} (oracle {np.round(sq_ref, 6)}), smallest gap {gaps:.2e}")
    b = _bound(r2, ev)
    np.testing.assert_allclose(sq, sq_ref, atol=4 * b * max(1.0, sq_ref.max()))
    if gaps > 1e-4:
        assert np.abs(_align(g, ref) - ref).max() < b
