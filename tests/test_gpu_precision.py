"""Sigma in every contraction precision (FP64 on the matrix cores or the FMA
kernel, FP32 and BF16x3 on the matrix cores) against the FP64 oracle, at
sizes that fit one 64x64 tile and at sizes whose symmetry blocks span several
tiles with a ragged tail (PPP chain L=12, bond sectors up to 88 states).

Tolerances (relative 2-norm error of the sigma block vector):
  FP64   1e-12: rounding of sums of O(10^3) terms at unit roundoff 1.1e-16.
  FP32   1e-5 : unit roundoff 6e-8 grown over two staged contractions whose
                inner lengths reach a few hundred (sqrt(K) growth, plus
                cancellation between channel contributions).
  BF16x3 1e-4 : the dropped lo*lo product and the rounding of lo are each
                about 2^-16 relative per product (1.5e-5), with the same
                growth as FP32."""
import numpy as np
import pytest

import synth
from oracle import fci, mpsvec

from synth import mps_arrays

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}


def _prec(lib, name):
    return {"fp64": lib.FP64, "fp32": lib.FP32, "bf16x3": lib.BF16X3}[name]


def _ctx(lib, L, Na, Nb, h, eri, mps):
    ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
    ctx.import_mps(*mps_arrays(mps))
    ctx.build_ops()
    return ctx


def _rel(out, ref):
    return float(np.linalg.norm(out - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("L,Na,Nb,M,seed", [(4, 2, 2, 8, 3), (6, 3, 3, 16, 11), (6, 2, 3, 12, 5)])
def test_low_precision_sigma_small(L, Na, Nb, M, seed, prec):
    import paper_1311_1646_amd as lib
    h, eri, _ = synth.random_integrals(L, seed=seed, K=8, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, M, seed=seed + 1)
    ctx = _ctx(lib, L, Na, Nb, h, eri, mps)
    dets, H = fci.hamiltonian(h, eri, 0.0, Na, Nb)
    rng = np.random.default_rng(seed)
    for w in (1, 2):
        for i in range(L - w + 1):
            P = mpsvec.site_basis(mps, dets, i) if w == 1 else mpsvec.two_site_basis(mps, dets, i)
            C = rng.normal(size=(3, P.shape[1]))
            ref = C @ mpsvec.heff(H, P).T
            kind = lib.SIGMA_ZEROTH_1SITE if w == 1 else lib.SIGMA_ZEROTH_2SITE
            out = ctx.sigma(i, torch.tensor(C, device="cuda"), kind=kind, prec=_prec(lib, prec)).cpu().numpy()
            err = _rel(out, ref)
            assert err < TOL[prec], (w, i, err)
    ctx.close()


@pytest.fixture(scope="module")
def ppp12():
    L, Na, Nb, M = 12, 3, 3, 400
    h, eri, _ = synth.ppp_integrals(L)
    mps = synth.random_mps(L, Na, Nb, M, seed=5)
    assert max(d for _, d in mps.bonds[6]) > 64   # blocks wider than one tile
    dets, H = fci.hamiltonian(h, eri, 0.0, Na, Nb)
    return L, Na, Nb, h, eri, mps, dets, H


@pytest.mark.parametrize("prec,fp64_gemm", [("fp64", "mfma"), ("fp64", "fma"), ("fp32", None), ("bf16x3", None)])
def test_multi_tile_sigma(ppp12, prec, fp64_gemm, monkeypatch):
    import paper_1311_1646_amd as lib
    L, Na, Nb, h, eri, mps, dets, H = ppp12
    if fp64_gemm:
        monkeypatch.setenv("DMRG_FP64_GEMM", fp64_gemm)
    ctx = _ctx(lib, L, Na, Nb, h, eri, mps)
    rng = np.random.default_rng(17)
    print(f"[multi-tile] prec={prec} gemm={fp64_gemm}", flush=True)
    for w, sites in ((1, (0, 4, 5, 6, 11)), (2, (5,))):
        kind = lib.SIGMA_ZEROTH_1SITE if w == 1 else lib.SIGMA_ZEROTH_2SITE
        for i in sites:
            _, n = ctx.layout(i, w)
            C = rng.normal(size=(4, n))
            ref = mpsvec.heff_apply(H, mps, dets, i, C, width=w)
            out = ctx.sigma(i, torch.tensor(C, device="cuda"), kind=kind, prec=_prec(lib, prec)).cpu().numpy()
            err = _rel(out, ref)
            print(f"  w={w} site={i} n={n} rel={err:.3e}", flush=True)
            assert err < TOL[prec], (w, i, err)
    ctx.close()


@pytest.mark.parametrize("shape", ["64x64", "128x64", "64x128", "128x128"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_every_tile_shape(ppp12, prec, shape, monkeypatch):
    # each matrix-core tile shape (where the batch folding allows it) on
    # blocks wider than 64 with a ragged edge
    import paper_1311_1646_amd as lib
    L, Na, Nb, h, eri, mps, dets, H = ppp12
    monkeypatch.setenv("DMRG_TILE_SHAPE", shape)
    ctx = _ctx(lib, L, Na, Nb, h, eri, mps)
    rng = np.random.default_rng(29)
    for w, i in ((1, 5), (1, 6), (2, 5)):
        kind = lib.SIGMA_ZEROTH_1SITE if w == 1 else lib.SIGMA_ZEROTH_2SITE
        _, n = ctx.layout(i, w)
        C = rng.normal(size=(3, n))
        ref = mpsvec.heff_apply(H, mps, dets, i, C, width=w)
        out = ctx.sigma(i, torch.tensor(C, device="cuda"), kind=kind, prec=_prec(lib, prec)).cpu().numpy()
        err = _rel(out, ref)
        assert err < TOL[prec], (shape, w, i, err)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_autotuned_shapes_keep_parity(ppp12, prec):
    # the autotuner's choice (any pair of stage shapes) leaves the sigma at
    # the precision's tolerance, at the tuned site and at others
    import paper_1311_1646_amd as lib
    L, Na, Nb, h, eri, mps, dets, H = ppp12
    ctx = _ctx(lib, L, Na, Nb, h, eri, mps)
    s1, s2, ms = ctx.autotune(5, 3, _prec(lib, prec))
    assert s1 in (-1, 0, 1, 2) and s2 in (-1, 0, 1, 2) and ms > 0
    rng = np.random.default_rng(31)
    for w, i in ((1, 5), (1, 3), (2, 6)):
        kind = lib.SIGMA_ZEROTH_1SITE if w == 1 else lib.SIGMA_ZEROTH_2SITE
        _, n = ctx.layout(i, w)
        C = rng.normal(size=(3, n))
        ref = mpsvec.heff_apply(H, mps, dets, i, C, width=w)
        out = ctx.sigma(i, torch.tensor(C, device="cuda"), kind=kind, prec=_prec(lib, prec)).cpu().numpy()
        err = _rel(out, ref)
        assert err < TOL[prec], (s1, s2, w, i, err)
    ctx.close()
