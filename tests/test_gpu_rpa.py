"""GPU parity of the DMRG-RPA sweep Davidson (dmrg_rpa_roots; Sec. II C eq.
dmrgrpa, Sec. III E eqs. reducedrpa and bmatrix) against the oracle's RPA in
the tangent space of the same MPS: a stationary truncated reference (one-site
DMRG on the CPU, where W is large: the lowest RPA root lies far below the TDA
one), with a small trial space so that the run restarts, in FP64 and in FP32
with FP64 polish; and an exact reference, where W vanishes and the RPA roots
are the FCI excitation energies."""
import numpy as np
import pytest

import synth
import stationary_reference
from oracle import fci, mpsvec, rpa
from synth import mps_arrays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stationary():
    L, Na, Nb, M, seed, n = 6, 3, 3, 10, 5, 3
    h, eri, _ = synth.random_integrals(L, seed=seed, K=L, diag_lo=-2, diag_hi=0)
    dets, H = fci.hamiltonian(h, eri, 0.0, Na, Nb)
    mps, e, sweeps = stationary_reference.onesite_ground(synth.random_mps(L, Na, Nb, M, seed), dets, H)
    g = stationary_reference.gradient_norm(mps, dets, H)
    e0, om_rpa, om_tda = rpa.rpa_roots(mps, dets, H, n)
    print(f"reference: E {e:.12f} after {sweeps} one-site sweeps, gradient {g:.2e}; oracle RPA "
          f"{np.round(om_rpa, 10).tolist()} TDA {np.round(om_tda, 10).tolist()}", flush=True)
    return (L, Na, Nb, h, eri, mps, n, om_rpa, om_tda)


def _gpu_rpa(case, prec, max_space, tol):
    import paper_1311_1646_amd as lib
    L, Na, Nb, h, eri, mps, n, _, _ = case
    ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
    ctx.import_mps(*mps_arrays(mps))
    ctx.build_ops(prec)
    return ctx.rpa_roots(n, max_iter=150, max_space=max_space, tol=tol, seed=3, prec=prec)


def test_rpa_roots_match_the_oracle_through_restarts(stationary):
    om, et, r2, it, conv = _gpu_rpa(stationary, 0, 24, 1e-11)
    om_rpa, om_tda = stationary[7], stationary[8]
    print(f"FP64 RPA {np.round(om, 10).tolist()} in {it} iterations, max r2 {r2.max():.2e}", flush=True)
    assert conv, (it, r2)
    np.testing.assert_allclose(om, om_rpa, atol=1e-8)
    assert om[0] < om_tda[0] - 0.1


def test_rpa_fp32_with_fp64_polish_matches_the_oracle(stationary):
    # FP32 zeroth-order pools (built by build_ops in FP32) bound the
    # excitation energies at ~1e-7 |E| whatever the polish does; the bound is
    # the excitation-energy tolerance of the low-precision runs, 1e-5 Eh
    # (measured 4.7e-7 Eh at |E| = 13 Eh)
    om, et, r2, it, conv = _gpu_rpa(stationary, 1, 0, 1e-10)
    d = np.abs(om - stationary[7]).max()
    print(f"FP32 RPA {np.round(om, 10).tolist()} in {it} iterations, max r2 {r2.max():.2e}, "
          f"|d omega| {d:.2e}", flush=True)
    assert conv, (it, r2)
    assert d <= 1e-5


def test_exact_reference_rpa_is_the_fci_spectrum():
    import paper_1311_1646_amd as lib
    L, Na, Nb, n = 5, 2, 2, 3
    h, eri, _ = synth.random_integrals(L, seed=31, K=5, diag_lo=-2, diag_hi=0)
    dets, H, w, vec = fci.fci(h, eri, 0.0, Na, Nb, nroots=n + 1)
    bonds, A = mpsvec.fci_to_mps(vec[:, 0], dets, L, Na, Nb)
    mps = synth.canonical_from_tensors(L, Na, Nb, bonds, A)
    ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
    ctx.import_mps(*mps_arrays(mps))
    ctx.build_ops(0)
    om, et, r2, it, conv = ctx.rpa_roots(n, max_iter=80, tol=1e-11, seed=3, prec=0)
    print(f"exact reference RPA {np.round(om, 10).tolist()} in {it} iterations", flush=True)
    assert conv, (it, r2)
    np.testing.assert_allclose(om, w[1:n + 1] - w[0], atol=1e-8)



@pytest.mark.timeout(300)
def test_rpa_at_full_bond_dimension_is_tda_and_fci_at_scale():
    # L=8, N=8 random integrals at M=256, the full space (exact bond
    # dimensions 1,4,16,64,256,...): the sweep's MPS is the FCI ground state,
    # a stationary reference with (H - E0) Psi0 = 0, so W vanishes and the
    # RPA roots are the TDA roots and the FCI excitations.  W vanishes here
    # only through cancellations inside correct bra-side first-order
    # operators (blocks up to 70 wide, both pair modes), so any error in
    # them shows.  The iteration times of both runs are printed.
    import paper_1311_1646_amd as lib
    p = synth.config(0)
    dets, H, w, _ = fci.fci(p.h, p.eri, p.ecore, p.Na, p.Nb, nroots=5)
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    e, dw, ok = ctx.sweep_ground([32, 128, 256, 256, 256], davidson_tol=1e-13, davidson_max_iter=80, seed=1)
    assert ok and abs(e - w[0]) < 1e-9
    n = 4
    om_t, _, r2_t, it_t, conv_t = ctx.tda_roots(n, max_iter=200, max_space=40, tol=1e-10, seed=3)
    st_t = ctx.stats()
    om_r, _, r2_r, it_r, conv_r = ctx.rpa_roots(n, max_iter=200, max_space=40, tol=1e-10, seed=3)
    st_r = ctx.stats()
    print(f"TDA {it_t} iterations {st_t['tda_total_ms'] / 1e3:.2f} s ({st_t['tda_total_ms'] / it_t:.1f} ms/it); "
          f"RPA {it_r} iterations {st_r['tda_total_ms'] / 1e3:.2f} s ({st_r['tda_total_ms'] / it_r:.1f} ms/it); "
          f"RPA - FCI {np.abs(om_r - (w[1:n + 1] - w[0])).max():.2e}", flush=True)
    assert conv_t and conv_r, (it_t, r2_t, it_r, r2_r)
    np.testing.assert_allclose(om_r, om_t, atol=1e-7)
    np.testing.assert_allclose(om_r, w[1:n + 1] - w[0], atol=1e-7)


def test_rpa_from_the_librarys_onesite_polished_ground_state():
    # two-site sweeps alone leave a truncated MPS off the stationary point of
    # its manifold; one-site sweeps (dmrg_sweep_params.onesite_sweeps) bring
    # the library's own ground state there, and its RPA roots then equal the
    # oracle's RPA of the exported MPS
    import paper_1311_1646_amd as lib
    from synth import mps_from_arrays
    L, Na, Nb, M, seed, n = 6, 3, 3, 10, 5, 3
    h, eri, _ = synth.random_integrals(L, seed=seed, K=L, diag_lo=-2, diag_hi=0)
    dets, H = fci.hamiltonian(h, eri, 0.0, Na, Nb)
    ctx2 = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
    e2, _, _ = ctx2.sweep_ground([M, M, M], davidson_tol=1e-14, davidson_max_iter=60, seed=1)
    g2 = stationary_reference.gradient_norm(mps_from_arrays(L, Na, Nb, *ctx2.export_mps()), dets, H)
    ctx1 = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
    e1, _, _ = ctx1.sweep_ground([M, M, M], davidson_tol=1e-14, davidson_max_iter=60, seed=1, onesite_sweeps=60)
    mps1 = mps_from_arrays(L, Na, Nb, *ctx1.export_mps())
    g1 = stationary_reference.gradient_norm(mps1, dets, H)
    print(f"two-site E {e2:.12f} gradient {g2:.2e}; + one-site sweeps E {e1:.12f} gradient {g1:.2e}", flush=True)
    assert e1 <= e2 + 1e-10
    assert g1 < 1e-5 and g1 < 1e-2 * g2
    e0, om_ref, om_tda = rpa.rpa_roots(mps1, dets, H, n)
    om, et, r2, it, conv = ctx1.rpa_roots(n, max_iter=150, tol=1e-11, seed=3, prec=0)
    print(f"RPA {np.round(om, 10).tolist()} oracle {np.round(om_ref, 10).tolist()} in {it} iterations", flush=True)
    assert conv, (it, r2)
    np.testing.assert_allclose(om, om_ref, atol=1e-8)
