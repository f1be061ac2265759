"""Checks at the full benchmark size (L=36, N=30, M=1000, 16 vectors at the
middle site, the launch configuration bench.py times), where the dense
oracle cannot run: properties that hold at any size.

* Hermiticity: G = C^T (H C) is symmetric for any vectors C.
* Energy gauge invariance: <C_i|H|C_i> of the mixed-canonical MPS is the
  same energy at every site (the one-site bases of all sites span the same
  state, with operators renormalized through every bond).
* Precision ladder: FP32 and BF16x3 sigmas agree with the FP64 sigma within
  the bounds derived in test_gpu_precision.
* One-site vs two-site: projecting the two-site sigma of C_i R_{i+1} back
  with R_{i+1} gives the one-site sigma of C_i.
* One DMRG-TDA iteration (16 roots): symmetric reduced matrices, positive
  definite S_R, FP32 Ritz values within the FP32 error of the FP64 ones."""
import numpy as np
import pytest

import synth

from synth import mps_arrays

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def big():
    import paper_1311_1646_amd as lib
    p = synth.config(4, M=1000)
    mps = synth.random_mps(p.L, p.Na, p.Nb, p.M, seed=4001)
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    ctx.import_mps(*mps_arrays(mps))
    ctx.build_ops()
    yield p, mps, ctx
    ctx.close()


def test_hermitian_at_full_size(big):
    import paper_1311_1646_amd as lib
    p, mps, ctx = big
    site = p.L // 2
    _, n = ctx.layout(site)
    g = torch.Generator(device="cuda").manual_seed(5)
    C = torch.randn(16, n, dtype=torch.float64, device="cuda", generator=g)
    for prec, tol in ((lib.FP64, 1e-12), (lib.FP32, 1e-5)):
        S = ctx.sigma(site, C, prec=prec)
        G = (C @ S.T).cpu().numpy()
        asym = np.abs(G - G.T).max() / np.abs(G).max()
        print(f"prec {prec}: asymmetry {asym:.2e}")
        assert asym < tol


def test_energy_same_at_every_site_full_size(big):
    p, mps, ctx = big
    E = []
    for i in range(p.L):
        c = torch.tensor(mps.flat("C", i)[None], device="cuda")
        s = ctx.sigma(i, c)
        E.append(float((c * s).sum() / (c * c).sum()))
    E = np.array(E)
    print(f"energy spread over sites {E.max() - E.min():.2e} (E = {E.mean():.8f})")
    assert E.max() - E.min() < 1e-9 * max(1.0, abs(E.mean()))


def test_precision_ladder_full_size(big):
    import paper_1311_1646_amd as lib
    p, mps, ctx = big
    site = p.L // 2
    _, n = ctx.layout(site)
    g = torch.Generator(device="cuda").manual_seed(6)
    C = torch.randn(16, n, dtype=torch.float64, device="cuda", generator=g)
    ref = ctx.sigma(site, C, prec=lib.FP64)
    for prec, tol in ((lib.FP32, 1e-5), (lib.BF16X3, 1e-4)):
        out = ctx.sigma(site, C, prec=prec)
        err = float(torch.linalg.norm(out - ref) / torch.linalg.norm(ref))
        print(f"prec {prec}: rel err {err:.2e}")
        assert err < tol


def test_two_site_sigma_projects_to_one_site_full_size(big):
    import paper_1311_1646_amd as lib
    p, mps, ctx = big
    i = p.L // 2
    b1, n1 = ctx.layout(i, 1)
    b2, n2 = ctx.layout(i, 2)
    br, _ = ctx.layout(i + 1, 1)
    R = mps.flat("R", i + 1)
    rblk = {(int(a), int(nn)): (int(c), int(r), int(cc), int(o)) for a, nn, c, r, cc, o in br}
    g = torch.Generator(device="cpu").manual_seed(7)
    C1 = torch.randn(n1, dtype=torch.float64, generator=g).numpy()
    # Psi(a, n1, n2, c) = sum_b C(a, n1, b) R(b, n2, c)
    o1 = {(int(a), int(nn)): (int(c), int(r), int(cc), int(o)) for a, nn, c, r, cc, o in b1}
    psi = np.zeros(n2)
    for a, nn, c, r, cc, o in b2:
        x, y = divmod(int(nn), 4)
        if (int(a), x) not in o1:
            continue
        b, ra, ca, oa = o1[(int(a), x)]
        if (b, y) not in rblk or rblk[(b, y)][0] != int(c):
            continue
        _, rr, cr, orr = rblk[(b, y)]
        psi[o:o + r * cc] = (C1[oa:oa + ra * ca].reshape(ra, ca) @ R[orr:orr + rr * cr].reshape(rr, cr)).ravel()
    s2 = ctx.sigma(i, torch.tensor(psi[None], device="cuda"), kind=lib.SIGMA_ZEROTH_2SITE).cpu().numpy()[0]
    s1 = ctx.sigma(i, torch.tensor(C1[None], device="cuda")).cpu().numpy()[0]
    # project: s1'(a, n1, b) = sum_{n2, c} s2(a, n1, n2, c) R(b, n2, c)^T
    proj = np.zeros(n1)
    for a, nn, c, r, cc, o in b2:
        x, y = divmod(int(nn), 4)
        if (int(a), x) not in o1:
            continue
        b, ra, ca, oa = o1[(int(a), x)]
        if (b, y) not in rblk or rblk[(b, y)][0] != int(c):
            continue
        _, rr, cr, orr = rblk[(b, y)]
        proj[oa:oa + ra * ca] += (s2[o:o + r * cc].reshape(r, cc) @ R[orr:orr + rr * cr].reshape(rr, cr).T).ravel()
    err = np.linalg.norm(proj - s1) / np.linalg.norm(s1)
    print(f"one-site vs projected two-site: {err:.2e}")
    assert err < 1e-12


@pytest.mark.timeout(600)
def test_tda_iteration_full_size_fp64_vs_fp32(big):
    # One DMRG-TDA Davidson iteration (16 roots, 32 trial vectors, the bench
    # launch) in FP64 and in FP32 from the same deterministic start: the
    # reduced matrices H_R, S_R of eq. eigs are symmetric with S_R positive
    # definite, and the Ritz values agree within the FP32 contraction error,
    # which enters H_R to first order: |d omega| < 1e-5 |E| (FP32 relative
    # error a few 2^-24 grown over sums of ~10^3 terms; measured 1.4e-7 |E|:
    # 6.5e-5 Eh at |E| = 474 Eh)
    p, mps, ctx = big
    res = {}
    for prec in (0, 1):
        om, et, r2, it, conv = ctx.tda_roots(16, max_iter=1, tol=0.0, seed=7, prec=prec, polish=False)
        HR, SR = ctx.tda_reduced()
        assert it == 1 and HR.shape == (32, 32)
        # rounding in H_R scales with |E| |x_mu| |x_nu| (norms from diag S_R)
        nrm = np.sqrt(np.abs(np.diag(SR)))
        scale = np.abs(et).max() * np.outer(nrm, nrm)
        asym = np.abs(HR - HR.T) / scale
        print(f"prec {prec}: max |H_R| {np.abs(HR).max():.3e}, max diag S_R {np.diag(SR).max():.3e}, "
              f"|E| {np.abs(et).max():.1f}, asymmetry {asym.max():.2e} of |E||x||x|")
        # FP64 measured 2.6e-16; FP32 contractions 2.0e-7 (FP32 rounding of
        # the sigma parts that enter H_R)
        assert asym.max() < {0: 1e-12, 1: 1e-5}[prec]
        assert np.abs(SR - SR.T).max() < 1e-12 * np.abs(SR).max()
        assert np.linalg.eigvalsh(0.5 * (SR + SR.T)).min() > 0
        assert np.all(np.isfinite(om)) and np.all(np.diff(om) >= 0)
        res[prec] = (om, et)
    d = np.abs(res[1][0] - res[0][0])
    print(f"one TDA iteration at M=1000: max |d omega| FP32 vs FP64 {d.max():.2e} Eh "
          f"(|E| ~ {np.abs(res[0][1]).max():.1f})")
    assert np.all(d < 1e-5 * np.abs(res[0][1]))
