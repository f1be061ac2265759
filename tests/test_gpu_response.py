"""GPU linear response (dmrg_response; Sec. II B, eqs. realresp and
imagresp) against the oracle's solve of the same equations in the explicit
tangent space.

The sweep solver is a Galerkin method in the trial space (as the TDA
Davidson), which converges steadily when both shifted operators H - (E0 -+
omega) are positive definite on the tangent space: a ground-state reference
(DMRG-optimized, so its TDA excitations are positive) and omega below the
lowest TDA excitation.  Those are the cases here, plus a small random
reference whose whole tangent space fits in the trial space."""
import numpy as np
import pytest

import synth
from oracle import fci, response, tda
from synth import mps_arrays, mps_from_arrays

pytestmark = pytest.mark.gpu


def _v(L, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(L, L))
    return 0.5 * (v + v.T)


def _check(ctx, mps, dets, H, v, Na, Nb, omegas, prec=0, rel=1e-8):
    V = response.onebody(v, Na, Nb)
    for om in omegas:
        cp, cm, r2, it, conv = ctx.response(v, om, max_iter=200, tol=1e-11, prec=prec)
        rp, rm = response.response(mps, dets, H, V, om)
        st = ctx.stats()
        print(f"prec {prec} omega {om:.4f}: chi+ {cp:.12f} ({rp:.12f}) chi- {cm:.12f} ({rm:.12f}) "
              f"in {it} iterations ({st['tda_polish_iters']} FP64)")
        assert conv, (om, it, r2)
        assert abs(cp - rp) < rel * max(1.0, abs(rp)), (om, cp, rp)
        assert abs(cm - rm) < rel * max(1.0, abs(rm)), (om, cm, rm)
        if prec != 0:
            assert st["tda_polish_iters"] >= 2


@pytest.fixture(scope="module")
def ground8():
    # config 0 (L=8, N=8, random dense integrals) ground state truncated to M=24
    import paper_1311_1646_amd as lib
    p = synth.config(0)
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    ctx.sweep_ground([16, 24, 24, 24], davidson_tol=1e-12, davidson_max_iter=60, seed=2)
    mps = mps_from_arrays(p.L, p.Na, p.Nb, *ctx.export_mps())
    dets, H = fci.hamiltonian(p.h, p.eri, p.ecore, p.Na, p.Nb)
    E0, roots = tda.tda_roots(mps, dets, H, 1)
    return p, ctx, mps, dets, H, roots[0] - E0


def test_ground_state_response_below_the_first_excitation(ground8):
    p, ctx, mps, dets, H, w1 = ground8
    assert w1 > 0.05
    # (closer to the pole the smaller eigenvalue of H - (E0 + omega) slows the
    # iteration: at 0.8 w1 the residual was 2.4e-5 after 150 iterations, chi
    # already within 2e-7 relative; the error of chi is second order in the
    # residual, |r|^2 over that eigenvalue)
    _check(ctx, mps, dets, H, _v(p.L, 5), p.Na, p.Nb, [0.0, 0.3 * w1, 0.6 * w1])


def test_ground_state_response_through_restarts(ground8):
    # a 10-vector space restarts every few iterations; the restarted space
    # keeps the current solutions x_pm themselves, so the solve still
    # converges to the oracle's
    p, ctx, mps, dets, H, w1 = ground8
    v = _v(p.L, 5)
    V = response.onebody(v, p.Na, p.Nb)
    om = 0.3 * w1
    cp, cm, r2, it, conv = ctx.response(v, om, max_iter=400, max_space=10, tol=1e-11)
    rp, rm = response.response(mps, dets, H, V, om)
    print(f"restarted (space 10): chi+ {cp:.12f} ({rp:.12f}) chi- {cm:.12f} ({rm:.12f}) in {it} iterations")
    assert conv, (it, r2)
    assert ctx.stats()["tda_space"] == 10
    assert abs(cp - rp) < 1e-8 * max(1.0, abs(rp)) and abs(cm - rm) < 1e-8 * max(1.0, abs(rm))


@pytest.mark.parametrize("prec", [1, 2])
def test_ground_state_response_low_precision_with_polish(ground8, prec):
    # FP32 / BF16x3 contractions finish with FP64 polish iterations, as in the TDA
    p, ctx, mps, dets, H, w1 = ground8
    _check(ctx, mps, dets, H, _v(p.L, 6), p.Na, p.Nb, [0.5 * w1], prec=prec)


def test_exact_reference_reproduces_the_fci_response():
    # full bond dimension (M=256 for L=8): the tangent space is the whole
    # complement of the ground state, so chi is the FCI sum over states.  The
    # GPU result equals the oracle's on the exported MPS to 1e-8; that equals
    # the FCI sum to the accuracy of the DMRG ground state itself (Davidson
    # residual ~3e-7, so |d Psi0| ~ 1e-6 and chi, linear in V Psi0, within
    # ~1e-6 relative): bound 1e-5
    import paper_1311_1646_amd as lib
    p = synth.config(0)
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    ctx.sweep_ground([32, 128, 256, 256, 256], davidson_tol=1e-13, davidson_max_iter=80, seed=1)
    mps = mps_from_arrays(p.L, p.Na, p.Nb, *ctx.export_mps())
    dets, H, w, vec = fci.fci(p.h, p.eri, p.ecore, p.Na, p.Nb, nroots=len(fci.determinants(p.L, p.Na, p.Nb)))
    v = _v(p.L, 8)
    V = response.onebody(v, p.Na, p.Nb)
    t = (vec[:, 1:].T @ (V @ vec[:, 0])) ** 2
    om = 0.5 * (w[1] - w[0])
    cp, cm, r2, it, conv = ctx.response(v, om, max_iter=200, tol=1e-11)
    rp, rm = response.response(mps, dets, H, V, om)
    ref_p = -np.sum(t / (w[1:] - w[0] + om))
    ref_m = -np.sum(t / (w[1:] - w[0] - om))
    print(f"exact: chi+ {cp:.10f} (oracle {rp:.10f}, FCI {ref_p:.10f}) chi- {cm:.10f} (oracle {rm:.10f}, "
          f"FCI {ref_m:.10f}) in {it} iterations")
    assert conv, (it, r2)
    assert abs(cp - rp) < 1e-8 * abs(rp) and abs(cm - rm) < 1e-8 * abs(rm)
    assert abs(rp - ref_p) < 1e-5 * abs(ref_p) and abs(rm - ref_m) < 1e-5 * abs(ref_m)


def test_small_random_reference_whole_tangent_space():
    # a random (not optimized) reference: indefinite shifted operators, but
    # the tangent space (dimension below the trial-space size) is spanned
    # exactly, so the Galerkin solution is the solve
    import paper_1311_1646_amd as lib
    L, Na, Nb, M, seed = 4, 2, 2, 6, 3
    h, eri, _ = synth.random_integrals(L, seed=seed, K=6, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, M, seed=seed + 1)
    ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
    ctx.import_mps(*mps_arrays(mps))
    ctx.build_ops()
    dets, H = fci.hamiltonian(h, eri, 0.0, Na, Nb)
    _check(ctx, mps, dets, H, _v(L, seed + 2), Na, Nb, [0.0, 0.21])


def test_response_argument_errors(ground8):
    import paper_1311_1646_amd as lib
    p, ctx, mps, dets, H, w1 = ground8
    v = _v(p.L, 5)
    with pytest.raises(lib.DMRGError, match="symmetric"):
        ctx.response(v + np.triu(np.ones_like(v), 1), 0.1)
    with pytest.raises(lib.DMRGError, match="finite"):
        ctx.response(v, float("nan"))
    with pytest.raises(ValueError):
        ctx.response(v[:3, :3], 0.1)
