"""GPU parity of the DMRG-TDA sweep Davidson against the oracle's plain
Rayleigh-Ritz in the MPS tangent space (reference projected out)."""
import numpy as np
import pytest

import synth
from oracle import fci, mpsvec, tda

from synth import mps_arrays

pytestmark = pytest.mark.gpu


def _run(L, Na, Nb, M, seed, nroots, K=6, tol=1e-12, max_iter=60, max_space=0, prec=0, stats=False, polish=True):
    import paper_1311_1646_amd as lib
    h, eri, _ = synth.random_integrals(L, seed=seed, K=K, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, M, seed=seed + 1)
    ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
    ctx.import_mps(*mps_arrays(mps))
    ctx.build_ops(prec)
    om, et, r2, it, conv = ctx.tda_roots(nroots, max_iter=max_iter, max_space=max_space, tol=tol, seed=3,
                                         prec=prec, polish=polish)
    st = ctx.stats()
    dets, H = fci.hamiltonian(h, eri, 0.0, Na, Nb)
    E0, ref = tda.tda_roots(mps, dets, H, nroots)
    if stats:
        return om, et, r2, it, conv, E0, ref, st
    return om, et, r2, it, conv, E0, ref


@pytest.mark.parametrize("L,Na,Nb,M,seed,n", [(4, 2, 2, 6, 3, 2), (6, 3, 3, 12, 11, 3), (6, 2, 3, 10, 5, 2)])
def test_tda_roots_match_tangent_space_rayleigh_ritz(L, Na, Nb, M, seed, n):
    om, et, r2, it, conv, E0, ref = _run(L, Na, Nb, M, seed, n)
    assert conv, (it, r2)
    np.testing.assert_allclose(et, ref, atol=1e-8)
    np.testing.assert_allclose(om, ref - E0, atol=1e-8)


def test_tda_config0_shape_four_roots():
    # L=8, N=8 random integrals as the correctness workload, truncated MPS
    om, et, r2, it, conv, E0, ref = _run(8, 4, 4, 24, 0, 4, K=16, tol=1e-11, max_space=40, max_iter=80)
    assert conv
    np.testing.assert_allclose(et, ref, atol=1e-8)
    np.testing.assert_allclose(om, ref - E0, atol=1e-8)


@pytest.mark.parametrize("prec", [1, 2])
def test_tda_low_precision_contractions_within_tolerance(prec):
    # FP32 / BF16x3 sigma and renormalization, FP64 Davidson, projections and
    # reduced matrices: excitation energies within 1e-5 Eh of the FP64 oracle
    # (the excitation-energy tolerance).  The eigenvalue error is first order
    # in the contraction error of the reduced matrices: ~1e-7 relative for
    # FP32 and ~2^-17 per split product for BF16x3 (measured up to 2.2e-5 Eh
    # here unpolished), in proportion to |E|.  Both runs therefore finish
    # with FP64 polish iterations once the residual reaches the floor of
    # their contractions; at least two run, and convergence is judged on the
    # FP64 residual.
    om, et, r2, it, conv, E0, ref, st = _run(8, 4, 4, 24, 0, 4, K=16, tol=1e-9, max_space=40, max_iter=80,
                                            prec=prec, stats=True)
    print(f"prec {prec}: |d omega| {np.abs(om - (ref - E0)).max():.2e} |d E| {np.abs(et - ref).max():.2e} "
          f"iterations {it} (fp64 polish {st['tda_polish_iters']})")
    assert conv, (it, r2)
    assert st["tda_polish_iters"] >= 2
    np.testing.assert_allclose(om, ref - E0, atol=1e-5)
    np.testing.assert_allclose(et, ref, atol=1e-5)


def test_bf16x3_without_polish_stays_within_split_precision_error():
    # the unpolished split precision alone: converged to its own residual
    # floor, within the 2^-17-per-product error estimate (4e-5 Eh here)
    om, et, r2, it, conv, E0, ref, st = _run(8, 4, 4, 24, 0, 4, K=16, tol=1e-7, max_space=40, max_iter=80,
                                            prec=2, stats=True, polish=False)
    print(f"bf16x3 unpolished: |d E| {np.abs(et - ref).max():.2e}")
    assert conv and st["tda_polish_iters"] == 0
    np.testing.assert_allclose(et, ref, atol=4e-5)


@pytest.mark.parametrize("prec", [1, 2])
def test_tda_low_precision_with_chunked_workspace(prec, monkeypatch):
    # A workspace budget of 300 elements per vector splits every contraction
    # of the sweep into many chunks, so the renormalizations of the
    # first-order sets (held in FP32 in these runs) accumulate their FP32
    # building blocks and destinations over several launches.  Same bound
    # as the unchunked low-precision test.
    monkeypatch.setenv("DMRG_T_BUDGET_PER_VEC", "300")
    om, et, r2, it, conv, E0, ref = _run(6, 3, 3, 12, 11, 3, tol=1e-9, max_iter=80, prec=prec)
    print(f"prec {prec} chunked: |d E| {np.abs(et - ref).max():.2e}")
    assert conv, (it, r2)
    np.testing.assert_allclose(et, ref, atol=1e-5)
    np.testing.assert_allclose(om, ref - E0, atol=1e-5)


def test_jsonl_metrics_log(tmp_path, monkeypatch):
    # DMRG_LOG_JSONL: one JSON line per ground-state sweep and per Davidson
    # iteration, consistent with what the calls return
    import json

    import paper_1311_1646_amd as lib
    path = tmp_path / "metrics.jsonl"
    monkeypatch.setenv("DMRG_LOG_JSONL", str(path))
    L, Na, Nb = 6, 3, 3
    h, eri, _ = synth.random_integrals(L, seed=11, K=6, diag_lo=-2, diag_hi=0)
    ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
    e, dw, _ = ctx.sweep_ground([16, 16, 16], davidson_tol=1e-12, davidson_max_iter=40, seed=1)
    om, et, r2, it, conv = ctx.tda_roots(2, max_iter=60, tol=1e-10, seed=3)
    rows = [json.loads(x) for x in path.read_text().splitlines()]
    sweeps = [r for r in rows if r["event"] == "ground_sweep"]
    iters = [r for r in rows if r["event"] == "tda_iteration"]
    assert [r["sweep"] for r in sweeps] == [0, 1, 2] and all(r["M"] == 16 for r in sweeps)
    assert abs(sweeps[-1]["energy"] - e) < 1e-6
    assert conv and [r["iteration"] for r in iters] == list(range(1, it + 1))
    assert iters[-1]["max_r2"] < 1e-10 and abs(iters[-1]["omega0"] - om[0]) < 1e-10
