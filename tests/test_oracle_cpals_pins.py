"""Pins of the oracle's CP-ALS compression (the paper's own low-rank step of
Algorithm 2, Section III-B; ALS settings of Section IV).  Each check is
independent of the oracle's unfolding and Khatri-Rao code: least-squares
solutions come from numpy.linalg.lstsq on design matrices built by einsum,
reconstructions from element sums."""
import itertools

import numpy as np
import pytest

from oracle import apg, cpals
from oracle.apg import TuckerData


def _lstsq_mode(X, U, n):
    """argmin_{U_n} ||X - [[U]]||_F with the other factors fixed, by lstsq on
    an explicit design matrix (rows: the other indices in C order)."""
    others = [m for m in range(3) if m != n]
    a, b = U[others[0]], U[others[1]]
    B = np.einsum("jr,kr->jkr", a, b).reshape(-1, a.shape[1])
    Xm = np.moveaxis(X, n, 0).reshape(X.shape[n], -1)
    sol, *_ = np.linalg.lstsq(B, Xm.T, rcond=None)
    return sol.T


def _brute_reconstruct(U):
    I = [u.shape[0] for u in U]
    R = U[0].shape[1]
    X = np.zeros(I)
    for i, j, k in itertools.product(*[range(d) for d in I]):
        X[i, j, k] = sum(U[0][i, r] * U[1][j, r] * U[2][k, r] for r in range(R))
    return X


def _problem(seed, dims=(7, 8, 9), R=3, noise=0.05):
    rng = np.random.default_rng(seed)
    T = [rng.random((d, R)) for d in dims]
    X = _brute_reconstruct(T)
    X = X + noise * rng.standard_normal(X.shape) * np.linalg.norm(X) / np.sqrt(X.size)
    U0 = [rng.random((d, R)) for d in dims]
    return X, U0


def test_one_iteration_is_three_sequential_least_squares_solves():
    X, U0 = _problem(1)
    want = [u.copy() for u in U0]
    for n in range(3):
        want[n] = _lstsq_mode(X, want, n)
    got = cpals.als_iteration(X, U0)
    for n in range(3):
        np.testing.assert_allclose(got[n], want[n], rtol=1e-9, atol=1e-12)


def test_relerr_matches_element_sum_and_never_increases():
    X, U0 = _problem(2, R=4)
    U, it, hist = cpals.cp_als(X, U0, eps=0.0, max_it=30)
    assert it == 30 and len(hist) == 31
    r = np.linalg.norm(X - _brute_reconstruct(U)) / np.linalg.norm(X)
    assert hist[-1] == pytest.approx(r, rel=1e-12)
    assert all(hist[k + 1] <= hist[k] * (1 + 1e-12) for k in range(30))


def test_rank_one_tensor_is_fitted_in_one_iteration():
    rng = np.random.default_rng(3)
    T = [rng.random((d, 1)) + 0.1 for d in (5, 6, 7)]
    X = _brute_reconstruct(T)
    U0 = [rng.random((d, 1)) + 0.1 for d in (5, 6, 7)]
    U, it, hist = cpals.cp_als(X, U0, eps=1e-4, max_it=200)
    assert hist[1] < 1e-14
    assert it == 2      # the second iteration changes RelErr by < eps


def test_noiseless_exact_rank_is_recovered():
    rng = np.random.default_rng(4)
    T = [rng.standard_normal((d, 3)) for d in (8, 9, 10)]
    X = _brute_reconstruct(T)
    U0 = [rng.standard_normal((d, 3)) for d in (8, 9, 10)]
    U, it, hist = cpals.cp_als(X, U0, eps=0.0, max_it=500)
    assert hist[-1] < 1e-8


@pytest.mark.parametrize("eps,max_it", [(1e-4, 200), (1e-2, 200), (0.0, 7)])
def test_stopping_rule(eps, max_it):
    X, U0 = _problem(5, R=3, noise=0.2)
    U, it, hist = cpals.cp_als(X, U0, eps=eps, max_it=max_it)
    assert len(hist) == it + 1
    first = next((k for k in range(1, len(hist)) if abs(hist[k] - hist[k - 1]) < eps), None)
    assert it == (first if first is not None else max_it)
    assert it <= max_it


def test_kruskal_as_tucker_reconstructs_and_feeds_lra_identities():
    X, U0 = _problem(6, dims=(4, 5, 3), R=3)
    U, _, _ = cpals.cp_als(X, U0, max_it=10)
    G, A = cpals.kruskal_as_tucker(U)
    Xt = _brute_reconstruct(U)
    D = TuckerData([G], [A])
    np.testing.assert_allclose(D.dense(0), Xt, rtol=1e-12, atol=1e-13)
    rng = np.random.default_rng(7)
    W = [rng.random((d, 2)) for d in (4, 5, 3)]
    for n in range(3):
        # element-sum MTTKRP of the reconstructed block
        Kb = np.zeros((Xt.shape[n], 2))
        for idx in itertools.product(*[range(d) for d in Xt.shape]):
            o = [m for m in range(3) if m != n]
            Kb[idx[n]] += Xt[idx] * W[o[0]][idx[o[0]]] * W[o[1]][idx[o[1]]]
        np.testing.assert_allclose(D.mttkrp(0, W, n), Kb, rtol=1e-11, atol=1e-12)
