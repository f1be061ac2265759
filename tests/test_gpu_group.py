"""Grouped sigma of many independent problems (dmrg_group_*): members with
different L, M and sites apply their zeroth-order sigma (Sec. III B, eq.
hzero_sb) in one launch per contraction stage, eagerly and replayed from a
HIP graph.  Each member's result is compared with its own dmrg_sigma (same
work lists; only the split of long contribution lists into segments may
differ, which changes the summation order) and, for members small enough,
with the oracle's dense effective Hamiltonian.  Every graph replay runs on
new input values in the same buffers and is checked against the eager
result of that replay's inputs (replays after the first included).

Tolerances (relative 2-norm): FP64 1e-12 against dmrg_sigma and the
oracle; FP32 1e-6 against the FP32 dmrg_sigma (summation order of FP32
partial sums) and 1e-5 against the oracle (as in the precision tests)."""
import numpy as np
import pytest

import synth
from oracle import fci, mpsvec
from synth import mps_arrays

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (L, n_alpha, n_beta, M, seed, site): several tiles and ragged blocks,
# different sizes in one launch
MEMBERS = [(6, 3, 3, 16, 11, 2), (8, 4, 4, 64, 21, 4), (7, 3, 4, 40, 33, 3), (5, 2, 3, 10, 7, 1),
           (8, 4, 4, 48, 45, 5), (10, 5, 5, 90, 51, 5)]


@pytest.fixture(scope="module")
def members():
    import paper_1311_1646_amd as lib
    out = []
    for L, Na, Nb, M, seed, site in MEMBERS:
        h, eri, _ = synth.random_integrals(L, seed=seed, K=8, diag_lo=-2, diag_hi=0)
        mps = synth.random_mps(L, Na, Nb, M, seed=seed + 1)
        ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
        ctx.import_mps(*mps_arrays(mps))
        ctx.build_ops()
        out.append((ctx, site, mps, h, eri, Na, Nb))
    yield out
    for m in out:
        m[0].close()


def _rel(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


@pytest.mark.parametrize("prec", [0, 1])
def test_group_matches_members_and_oracle(members, prec):
    import paper_1311_1646_amd as lib
    nvec = 3
    ctxs = [m[0] for m in members]
    sites = [m[1] for m in members]
    g = lib.Group(ctxs, sites, nvec, prec=prec)
    gen = torch.Generator(device="cuda").manual_seed(5)
    Cs = [torch.randn(nvec, c.size(i), dtype=torch.float64, device="cuda", generator=gen) for c, i in zip(ctxs, sites)]
    outs = [torch.empty_like(C) for C in Cs]
    tol = {0: 1e-12, 1: 1e-6}[prec]
    for step in range(4):  # eager, eager (first graph call builds lists), capture, replay
        for C in Cs:
            C.normal_(generator=gen)
        g.sigma(Cs, outs, graph=step > 0)
        torch.cuda.synchronize()
        print(f"[group] prec={prec} step={step} {g.stats()}", flush=True)
        for c, i, C, O in zip(ctxs, sites, Cs, outs):
            ref = c.sigma(i, C, prec=prec)
            assert _rel(O, ref) < tol, (step, i, _rel(O, ref))
    st = g.stats()
    assert st["graph_nodes"] >= st["launches"] >= 3
    # oracle for the members whose FCI space is small
    for (c, i, mps, h, eri, Na, Nb), C, O in zip(members, Cs, outs):
        if mps.L > 8:
            continue
        dets, H = fci.hamiltonian(h, eri, 0.0, Na, Nb)
        want = C.cpu().numpy() @ mpsvec.heff(H, mpsvec.site_basis(mps, dets, i)).T
        err = np.linalg.norm(O.cpu().numpy() - want) / np.linalg.norm(want)
        assert err < {0: 1e-12, 1: 1e-5}[prec], (i, err)
    # new buffers: only the base tables are uploaded again, the graph is reused
    Cs2 = [C.clone() * 0.5 for C in Cs]
    outs2 = [torch.empty_like(C) for C in Cs2]
    g.sigma(Cs2, outs2, graph=True)
    torch.cuda.synchronize()
    for O, O2 in zip(outs, outs2):
        assert _rel(O2, 0.5 * O) < tol
    g.close()


def test_group_rejects_changed_member(members):
    import paper_1311_1646_amd as lib
    ctxs = [m[0] for m in members[:2]]
    sites = [m[1] for m in members[:2]]
    g = lib.Group(ctxs, sites, 1, prec=0)
    Cs = [torch.ones(1, c.size(i), dtype=torch.float64, device="cuda") for c, i in zip(ctxs, sites)]
    outs = [torch.empty_like(C) for C in Cs]
    g.sigma(Cs, outs, graph=False)
    ctxs[1].build_ops()  # new operator pools: the group's pointers are stale
    with pytest.raises(lib.DMRGError) as e:
        g.sigma(Cs, outs, graph=False)
    assert e.value.code == -6
    g.close()
