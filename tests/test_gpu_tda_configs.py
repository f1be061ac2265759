"""DMRG-TDA converged at the two molecular-size workloads (Sec. IV): the PPP
polyene chain (L=24, N=24, M=256, six roots) and the dense water-shaped
Hamiltonian (L=24, N=10, M=500, eight roots), each after a ground-state sweep
to M.  FP64 contractions against FP32 / BF16x3 ones, which finish with FP64
polish iterations: the excitation energies agree within 1e-5 Eh, the reduced
matrices H_R and S_R of eq. eigs are symmetric with S_R positive definite,
and the residual falls steadily once the roots are located."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-7  # max over roots of sum_i |r_i|^2 at convergence


def _ground(cfg):
    import paper_1311_1646_amd as lib
    p = synth.config(cfg)
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    e, dw, _ = ctx.sweep_ground([p.M // 4, p.M // 2, p.M, p.M], davidson_tol=1e-10, davidson_max_iter=30, seed=1)
    print(f"{p.name}: ground {e:.10f} discarded weight {dw:.2e}", flush=True)
    return p, ctx


def _tda(p, ctx, prec):
    om, et, r2, it, conv = ctx.tda_roots(p.nroots, max_iter=150, tol=TOL, seed=3, prec=prec, verbose=1)
    st = ctx.stats()
    HR, SR = ctx.tda_reduced()
    print(f"{p.name} prec {prec}: converged {conv} in {it} iterations ({st['tda_polish_iters']} FP64 polish), "
          f"{st['tda_total_ms'] / 1e3:.1f} s, omega {np.round(om, 8).tolist()}", flush=True)
    return om, r2, it, conv, st, HR, SR


def _check_run(om, r2, it, conv, st, HR, SR, prec):
    assert conv, (it, r2)
    assert np.all(np.asarray(r2) < TOL)
    assert np.all(np.diff(om) >= 0) and om[0] > 0
    # eq. eigs: both reduced matrices are symmetric, S_R is a Gram matrix
    scale = np.abs(HR).max()
    np.testing.assert_allclose(HR, HR.T, atol=1e-10 * scale)
    np.testing.assert_allclose(SR, SR.T, atol=1e-12)
    assert np.linalg.eigvalsh(0.5 * (SR + SR.T)).min() > 0
    # residual decay: after the residual first drops below 1e-2 (the roots
    # located), the minimum over each window of eight iterations falls
    hist = np.asarray(st["tda_r2_hist"])
    assert len(hist) == it and hist[-1] < TOL
    start = int(np.argmax(hist < 1e-2))
    mins = [hist[k:k + 8].min() for k in range(start, len(hist), 8)]
    assert all(b <= a for a, b in zip(mins, mins[1:])), mins
    if prec != 0:
        assert st["tda_polish_iters"] >= 2
    # the default space (64 trial vectors) fits next to these workloads
    assert st["tda_space"] == 64


@pytest.fixture(scope="module")
def ppp():
    return _ground(1)


@pytest.fixture(scope="module")
def dense():
    return _ground(2)


@pytest.mark.timeout(600)
def test_ppp_chain_fp64_fp32_bf16x3_agree(ppp):
    p, ctx = ppp
    res = {prec: _tda(p, ctx, prec) for prec in (0, 1, 2)}
    for prec, r in res.items():
        _check_run(*r, prec)
    for prec in (1, 2):
        d = np.abs(res[prec][0] - res[0][0]).max()
        print(f"PPP |d omega| prec {prec} vs FP64: {d:.2e}")
        assert d <= 1e-5


@pytest.mark.timeout(900)
def test_dense_water_shaped_fp64_and_bf16x3_agree(dense):
    p, ctx = dense
    r64 = _tda(p, ctx, 0)
    _check_run(*r64, 0)
    r3 = _tda(p, ctx, 2)
    _check_run(*r3, 2)
    d = np.abs(r3[0] - r64[0]).max()
    print(f"dense |d omega| BF16x3 vs FP64: {d:.2e}")
    assert d <= 1e-5
