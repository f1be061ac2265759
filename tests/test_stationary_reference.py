"""The one-site DMRG helper that builds the stationary references of the RPA
GPU tests (tests/stationary_reference.py): it ends at a stationary point of
the energy on its fixed-bond-dimension MPS manifold (gradient measured with
the oracle's tangent space), its energy is <Psi|H|Psi> of the returned MPS,
and it is variational (above the FCI ground energy, below the energy of the
random start)."""
import numpy as np

import stationary_reference
import synth
from oracle import fci, mpsvec


def test_onesite_dmrg_reaches_a_stationary_point():
    L, Na, Nb, M, seed = 6, 3, 3, 10, 5
    h, eri, _ = synth.random_integrals(L, seed=seed, K=L, diag_lo=-2, diag_hi=0)
    dets, H, w, _ = fci.fci(h, eri, 0.0, Na, Nb, nroots=1)
    start = synth.random_mps(L, Na, Nb, M, seed)
    psi = mpsvec.mps_to_fci(start, dets)
    e_start = float(psi @ (H @ psi) / (psi @ psi))
    mps, e, sweeps = stationary_reference.onesite_ground(start, dets, H)
    psi = mpsvec.mps_to_fci(mps, dets)
    assert abs(float(psi @ (H @ psi) / (psi @ psi)) - e) < 1e-10
    assert w[0] - 1e-10 <= e < e_start
    g0 = stationary_reference.gradient_norm(start, dets, H)
    g = stationary_reference.gradient_norm(mps, dets, H)
    assert g < 1e-6 and g < 1e-4 * g0, (g0, g, sweeps)
