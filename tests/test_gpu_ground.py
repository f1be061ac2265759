"""GPU two-site ground-state DMRG: exactness at the full bond dimension
(energy = FCI, DMRG-TDA roots = FCI excited roots), the variational bound and
energy/gauge consistency of the returned MPS at truncated M, and the TDA on
that MPS against the oracle's tangent-space Rayleigh-Ritz."""
import numpy as np
import pytest

import synth
from oracle import fci, mpsvec, tda

from synth import mps_from_arrays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def config0():
    p = synth.config(0)
    dets, H, w, _ = fci.fci(p.h, p.eri, p.ecore, p.Na, p.Nb, nroots=5)
    return p, dets, H, w


def test_full_bond_dimension_reproduces_fci(config0):
    # L=8, N=8: exact bond dimensions 1,4,16,64,256,64,16,4,1, so M=256 is the
    # full space and DMRG, then DMRG-TDA, are exact (ground and 4 excitations)
    import paper_1311_1646_amd as lib
    p, dets, H, w = config0
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    e, dw, ok = ctx.sweep_ground([32, 128, 256, 256, 256], davidson_tol=1e-13, davidson_max_iter=80, seed=1)
    assert ok
    assert abs(e - w[0]) < 1e-9, (e, w[0])
    om, et, r2, it, conv = ctx.tda_roots(4, max_iter=200, max_space=40, tol=1e-10, seed=3)
    print(f"full-space TDA: {it} iterations, |r|^2 {r2}, omega - exact {om - (w[1:5] - w[0])}")
    assert conv, (it, r2)
    np.testing.assert_allclose(om, w[1:5] - w[0], atol=1e-7)


def test_truncated_sweep_is_variational_and_consistent(config0):
    import paper_1311_1646_amd as lib
    p, dets, H, w = config0
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    e, dw, ok = ctx.sweep_ground([16, 24, 24, 24], davidson_tol=1e-12, davidson_max_iter=60, seed=2)
    assert e > w[0] - 1e-10
    mps = mps_from_arrays(p.L, p.Na, p.Nb, *ctx.export_mps())
    assert max(d for b in mps.bonds for _, d in b) <= 24
    psi = mpsvec.mps_to_fci(mps, dets)
    assert abs(psi @ psi - 1) < 1e-10
    assert abs(mpsvec.energy(H, psi) - e) < 1e-9
    # the same state with the centre at every site (L C R gauge relations)
    for i in range(p.L):
        np.testing.assert_allclose(mpsvec.mps_to_fci(mps, dets, site=i), psi, atol=1e-10)
    E0, ref = tda.tda_roots(mps, dets, H, 3)
    om, et, r2, it, conv = ctx.tda_roots(3, max_iter=80, max_space=24, tol=1e-11, seed=3)
    assert conv
    np.testing.assert_allclose(et, ref, atol=1e-8)


@pytest.mark.parametrize("prec", [1, 2])
def test_low_precision_sweep_meets_ground_energy_tolerance(config0, prec):
    # FP32 or BF16x3 sigma and renormalization (BF16x3 builds the zeroth-order
    # pools in FP32), FP64 Davidson / SVD and the final energy evaluated in
    # FP64: |E - E_FCI| <= 1e-6 Eh at the full bond dimension (the north-star
    # ground-energy tolerance).  The energy is variational in the state, so
    # a contraction error eps in the local solves enters it at O(eps^2).
    import paper_1311_1646_amd as lib
    p, dets, H, w = config0
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    e, dw, ok = ctx.sweep_ground([64, 256, 256, 256], davidson_tol=1e-10, davidson_max_iter=60, seed=1,
                                 prec=prec)
    print(f"prec {prec} ground: E - E_FCI = {e - w[0]:.2e}")
    assert abs(e - w[0]) < 1e-6
