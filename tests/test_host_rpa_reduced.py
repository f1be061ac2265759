"""The reduced DMRG-RPA problem of Sec. III E eq. reducedrpa, solved on the
host by the library (dmrg_rpa_reduced, no device), against numpy's
eigenvalues of the full RPA matrix [[A, W], [-W, -A]] when the trial vectors
span the whole space (with redundant columns, so that S_R is singular), and
against the RPA equations themselves for the returned amplitudes."""
import numpy as np
import pytest

import paper_1311_1646_amd as lib


def _stable_problem(n, seed, wscale=0.4):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q @ np.diag(rng.uniform(1.0, 3.0, n)) @ Q.T
    W = rng.normal(size=(n, n))
    W = 0.5 * (W + W.T)
    W *= wscale / np.linalg.norm(W, 2)
    return A, W


def _reduced(A, W, U, e0):
    H = A + e0 * np.eye(A.shape[0])
    return U.T @ H @ U, U.T @ U, U.T @ W @ U


def test_full_span_with_redundant_vectors_gives_the_full_rpa_roots():
    n, e0 = 12, -7.5
    A, W = _stable_problem(n, 3)
    rng = np.random.default_rng(4)
    U = rng.normal(size=(n, n))
    U = np.concatenate([U, U[:, :3] @ rng.normal(size=(3, 3))], axis=1)  # three dependent columns
    HR, SR, WR = _reduced(A, W, U, e0)
    om, a, b, rank = lib.rpa_reduced(HR, SR, WR, e0, 5)
    assert rank == n
    ref = np.sort(np.linalg.eigvals(np.block([[A, W], [-W, -A]])).real)[n:]
    np.testing.assert_allclose(om, ref[:5], rtol=1e-11)
    X, Y = U @ a, U @ b
    for k in range(5):
        np.testing.assert_allclose(A @ X[:, k] + W @ Y[:, k], om[k] * X[:, k], atol=1e-9)
        np.testing.assert_allclose(W @ X[:, k] + A @ Y[:, k], -om[k] * Y[:, k], atol=1e-9)
        assert abs(X[:, k] @ X[:, k] - Y[:, k] @ Y[:, k] - 1.0) < 1e-10


def test_subspace_roots_bound_the_full_ones_and_w_zero_is_tda():
    n, e0 = 10, 1.25
    A, W = _stable_problem(n, 8)
    rng = np.random.default_rng(9)
    U = rng.normal(size=(n, 6))
    HR, SR, WR = _reduced(A, W, U, e0)
    om, a, b, rank = lib.rpa_reduced(HR, SR, WR, e0, 3)
    assert rank == 6
    # the same problem through numpy in an S_R-orthonormal basis of the span
    s, V = np.linalg.eigh(SR)
    T = V / np.sqrt(s)
    Ap = T.T @ (HR - e0 * SR) @ T
    Wp = T.T @ WR @ T
    ref = np.sort(np.linalg.eigvals(np.block([[Ap, Wp], [-Wp, -Ap]])).real)[6:]
    np.testing.assert_allclose(om, ref[:3], rtol=1e-11)
    # with W = 0 the roots are the TDA (generalized symmetric) eigenvalues
    om0, a0, b0, _ = lib.rpa_reduced(HR, SR, np.zeros_like(WR), e0, 3)
    np.testing.assert_allclose(om0, np.linalg.eigvalsh(Ap)[:3], rtol=1e-11)
    assert np.abs(b0).max() < 1e-10


def test_unstable_reference_is_reported():
    n, e0 = 6, 0.0
    A, W = _stable_problem(n, 5, wscale=0.4)
    A = A - 1.5 * np.eye(n)  # an A - W with negative directions
    U = np.eye(n)
    HR, SR, WR = _reduced(A, W, U, e0)
    with pytest.raises(lib.DMRGError):
        lib.rpa_reduced(HR, SR, WR, e0, 2)
