"""Host-side checks of the channel factorization of H (no GPU): the site
operators contracted densely must reproduce the brute-force Fock-space
Hamiltonian of the oracle, in both contraction directions and with one- and
two-site dots (this covers the normal -> complementary switch)."""
import numpy as np
import pytest

import synth
from oracle import fock

lib = pytest.importorskip("paper_1311_1646_amd")


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_factorized_hamiltonian_equals_fock_space(L):
    h, eri, _ = synth.random_integrals(L, seed=40 + L, K=4, diag_lo=-1, diag_hi=0.5)
    ctx = lib.Context(L, L // 2, L - L // 2, h, eri, 0.25, device=-1)
    Hf = fock.fock_hamiltonian(h, eri, 0.25)
    for wide in [-1] + list(range(L - 1)):
        for right in (False, True):
            Hd = ctx.debug_mpo_dense(wide, right)
            assert np.abs(Hd - Hf).max() < 1e-12, (wide, right)


def test_ppp_screening_drops_pair_channels():
    # Density-density interactions have no pair operators with both indices on
    # one side of a cut, so only O(L) channels survive per bond.
    p = synth.config(1)
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, 0.0, device=-1)
    assert max(ctx.num_channels(b) for b in range(p.L + 1)) <= 2 * p.L


def test_channel_count_dense_integrals():
    # generic integrals: 2 + 4|L| + ... ~ O(k^2) channels at mid-chain
    p = synth.config(0)
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, 0.0, device=-1)
    n = [ctx.num_channels(b) for b in range(p.L + 1)]
    assert n[0] == 1 and n[-1] == 1
    assert n[4] > n[1]


def test_invalid_arguments_raise():
    h = np.zeros((4, 4))
    eri = np.zeros((4,) * 4)
    with pytest.raises(lib.DMRGError):
        lib.Context(1, 1, 0, h[:1, :1], eri[:1, :1, :1, :1], device=-1)
    ctx = lib.Context(4, 2, 2, h, eri, device=-1)
    with pytest.raises(lib.DMRGError):
        ctx.debug_mpo_dense(7)
    with pytest.raises(lib.DMRGError):
        ctx.build_ops()   # host-only context refuses device work


@pytest.mark.parametrize("L", [3, 4])
def test_nonsymmetric_one_body_operator_factorizes_exactly(L):
    # the transition densities use contexts that hold a single E_pq (or any
    # non-symmetric one-body matrix): its channel factorization must equal the
    # Fock-space operator sum_pq v_pq a+_p a_q (spin-summed)
    rng = np.random.default_rng(L)
    v = rng.normal(size=(L, L))
    zero = np.zeros((L,) * 4)
    cases = [v]
    for p, q in ((0, L - 1), (L - 1, 0), (1, 1)):
        e = np.zeros((L, L))
        e[p, q] = 1.0
        cases.append(e)
    for m in cases:
        ctx = lib.Context(L, L // 2, L - L // 2, m, zero, 0.0, device=-1)
        Hf = fock.fock_hamiltonian(m, zero, 0.0)
        for wide in [-1] + list(range(L - 1)):
            for right in (False, True):
                assert np.abs(ctx.debug_mpo_dense(wide, right) - Hf).max() < 1e-12
