"""GPU parity of the sigma vector and its diagonal against the FP64 oracle's
dense effective Hamiltonian P^T H P.  The renormalized block operators are
not exported; they are pinned through the sigma at every site, which
contracts the left set of bond i with the right set of bond i+1."""
import numpy as np
import pytest

import synth
from oracle import fci, mpsvec

from synth import mps_arrays

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _setup(L, Na, Nb, M, seed, K=8, ecore=0.0):
    import paper_1311_1646_amd as lib
    h, eri, _ = synth.random_integrals(L, seed=seed, K=K, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, M, seed=seed + 1)
    ctx = lib.Context(L, Na, Nb, h, eri, ecore, device=0)
    ctx.import_mps(*mps_arrays(mps))
    ctx.build_ops()
    dets, H = fci.hamiltonian(h, eri, ecore, Na, Nb)
    return ctx, mps, dets, H


CASES = [(4, 2, 2, 8, 3), (6, 3, 3, 16, 11), (6, 2, 3, 12, 5), (8, 4, 4, 64, 21)]


@pytest.mark.parametrize("L,Na,Nb,M,seed", CASES)
def test_one_site_sigma_matches_dense_heff(L, Na, Nb, M, seed):
    ctx, mps, dets, H = _setup(L, Na, Nb, M, seed, ecore=0.37)
    rng = np.random.default_rng(seed)
    for i in range(L):
        P = mpsvec.site_basis(mps, dets, i)
        He = mpsvec.heff(H, P)
        C = rng.normal(size=(3, P.shape[1]))
        ref = C @ He.T
        out = ctx.sigma(i, torch.tensor(C, device="cuda")).cpu().numpy()
        err = np.abs(out - ref).max() / max(np.abs(ref).max(), 1.0)
        assert err < 1e-12, (i, err)


@pytest.mark.parametrize("L,Na,Nb,M,seed", CASES[:3])
def test_two_site_sigma_matches_dense_heff(L, Na, Nb, M, seed):
    import paper_1311_1646_amd as lib
    ctx, mps, dets, H = _setup(L, Na, Nb, M, seed)
    rng = np.random.default_rng(seed + 100)
    for i in range(L - 1):
        P = mpsvec.two_site_basis(mps, dets, i)
        He = mpsvec.heff(H, P)
        C = rng.normal(size=(2, P.shape[1]))
        out = ctx.sigma(i, torch.tensor(C, device="cuda"), kind=lib.SIGMA_ZEROTH_2SITE).cpu().numpy()
        ref = C @ He.T
        err = np.abs(out - ref).max() / max(np.abs(ref).max(), 1.0)
        assert err < 1e-12, (i, err)


@pytest.mark.parametrize("L,Na,Nb,M,seed", CASES[1:])
def test_diagonal_matches_dense_heff(L, Na, Nb, M, seed):
    ctx, mps, dets, H = _setup(L, Na, Nb, M, seed)
    for i in range(L):
        P = mpsvec.site_basis(mps, dets, i)
        ref = np.diag(mpsvec.heff(H, P))
        out = ctx.diag(i).cpu().numpy()
        assert np.abs(out - ref).max() < 1e-12 * max(1, np.abs(ref).max())


def test_energy_equal_at_every_site_and_hermitian():
    L, Na, Nb = 8, 4, 4
    ctx, mps, dets, H = _setup(L, Na, Nb, 40, seed=77)
    psi = mpsvec.mps_to_fci(mps, dets)
    E = mpsvec.energy(H, psi)
    rng = np.random.default_rng(1)
    for i in range(L):
        c = mps.flat("C", i)
        s = ctx.sigma(i, torch.tensor(c[None], device="cuda")).cpu().numpy()[0]
        assert abs(c @ s - E) < 1e-11
        x, y = rng.normal(size=(2, c.size))
        sx, sy = ctx.sigma(i, torch.tensor(np.stack([x, y]), device="cuda")).cpu().numpy()
        assert abs(x @ sy - y @ sx) < 1e-11 * (1 + abs(x @ sy))


def test_full_space_sigma_spectrum_is_fci():
    # untruncated bonds: H_eff at any site has exactly the FCI spectrum
    L, Na, Nb = 5, 2, 3
    ctx, mps, dets, H = _setup(L, Na, Nb, 10 ** 6, seed=9)
    w = np.linalg.eigvalsh(H.toarray())
    n = len(dets)
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    Hs = ctx.sigma(2, eye).cpu().numpy()
    np.testing.assert_allclose(np.linalg.eigvalsh(0.5 * (Hs + Hs.T)), w, atol=1e-10)


def test_renormalize_call_reproduces_build_ops():
    import paper_1311_1646_amd as lib
    L, Na, Nb = 6, 3, 3
    ctx, mps, dets, H = _setup(L, Na, Nb, 16, seed=4)
    C = torch.tensor(np.random.default_rng(3).normal(size=(1, mps.site_size(3))), device="cuda")
    before = ctx.sigma(3, C).clone()
    ctx.renormalize(2, lib.DIR_LEFT)
    ctx.renormalize(4, lib.DIR_RIGHT)
    after = ctx.sigma(3, C)
    assert torch.equal(before, after)


def test_chunked_workspace_gives_identical_sigma_at_every_site(monkeypatch):
    # a tiny workspace budget splits every contraction (the renormalizations
    # of the operator build and the sigmas) into many chunks; the sigma at
    # every site, which reads every operator set, must equal the unchunked
    # one (the summation order within an output block may differ: 1e-13)
    import paper_1311_1646_amd as lib
    L, Na, Nb = 6, 3, 3
    h, eri, _ = synth.random_integrals(L, seed=12, K=6, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, 16, seed=13)
    outs = []
    for budget in (None, "300"):
        if budget:
            monkeypatch.setenv("DMRG_T_BUDGET_PER_VEC", budget)
        ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
        ctx.import_mps(*mps_arrays(mps))
        ctx.build_ops()
        rng = np.random.default_rng(0)
        per_site = []
        for i in range(L):
            C = torch.tensor(rng.normal(size=(3, mps.site_size(i))), device="cuda")
            per_site.append(ctx.sigma(i, C).cpu().numpy())
        outs.append(per_site)
        ctx.close()
    for i in range(L):
        a, b = outs[0][i], outs[1][i]
        assert np.abs(a - b).max() < 1e-13 * np.abs(a).max(), i


def test_plans_built_on_threads_give_identical_results(monkeypatch):
    # the contraction plans of build_ops and of the TDA sweeps are built on a
    # pool of host threads; built on one thread they must give bit-identical
    # sigmas and TDA roots
    import paper_1311_1646_amd as lib
    L, Na, Nb = 8, 4, 4
    h, eri, _ = synth.random_integrals(L, seed=21, K=8, diag_lo=-2, diag_hi=0)
    mps = synth.random_mps(L, Na, Nb, 48, seed=22)
    res = []
    for threads in ("1", "16"):
        monkeypatch.setenv("DMRG_PLAN_THREADS", threads)
        ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
        ctx.import_mps(*mps_arrays(mps))
        ctx.build_ops()
        rng = np.random.default_rng(1)
        sig = []
        for i in range(L):
            C = torch.tensor(rng.normal(size=(2, mps.site_size(i))), device="cuda")
            sig.append(ctx.sigma(i, C).cpu().numpy())
        om, et, r2, it, conv = ctx.tda_roots(2, max_iter=40, tol=1e-10, seed=3)
        res.append((sig, om, it))
        ctx.close()
    for a, b in zip(res[0][0], res[1][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(res[0][1], res[1][1]) and res[0][2] == res[1][2]
