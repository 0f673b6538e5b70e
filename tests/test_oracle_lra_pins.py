"""Pins of the oracle's compression (truncated HOSVD) and of the low-rank
gradient identities of Section III-B (eq. eqlrag / eqlrau)."""
import itertools

import numpy as np
import pytest
import scipy.linalg

from oracle import apg, tucker
from oracle.apg import DenseData, Options, TuckerData
import synth

from test_oracle_pins import brute_mttkrp, brute_core_term


def brute_tucker(G, A):
    I = [a.shape[0] for a in A]
    X = np.zeros(I)
    for i, j, k in itertools.product(*[range(d) for d in I]):
        v = 0.0
        for a, b, c in itertools.product(*[range(d) for d in G.shape]):
            v += G[a, b, c] * A[0][i, a] * A[1][j, b] * A[2][k, c]
        X[i, j, k] = v
    return X


def test_thosvd_bases_orthonormal_and_norm_preserved():
    rng = np.random.default_rng(2)
    X = rng.random((7, 6, 5))
    G, A, ev = tucker.thosvd(X, (4, 3, 5))
    for n, An in enumerate(A):
        np.testing.assert_allclose(An.T @ An, np.eye(An.shape[1]), atol=1e-13)
    Xt = brute_tucker(G, A)
    assert np.linalg.norm(Xt) == pytest.approx(np.linalg.norm(G), rel=1e-13)
    # De Lathauwer et al. 2000: ||X - X~||^2 <= sum_n sum_{j > J_n} sigma_j^(n)^2
    bound = 0.0
    for n, J in enumerate((4, 3, 5)):
        s = scipy.linalg.svdvals(apg.unfold(X, n))
        bound += np.sum(s[J:] ** 2)
    assert np.linalg.norm(X - Xt) ** 2 <= bound * (1 + 1e-12)


def test_thosvd_bases_are_leading_left_singular_vectors():
    rng = np.random.default_rng(9)
    X = rng.random((6, 5, 4))
    _, A, ev = tucker.thosvd(X, (3, 3, 2))
    for n in range(3):
        Uu, s, _ = scipy.linalg.svd(apg.unfold(X, n), full_matrices=False)
        J = A[n].shape[1]
        np.testing.assert_allclose(ev[n], s[:J] ** 2, rtol=1e-11)
        # same vectors up to sign; the sign rule makes the largest entry positive
        for j in range(J):
            v = Uu[:, j] * np.sign(Uu[np.argmax(np.abs(Uu[:, j])), j])
            np.testing.assert_allclose(A[n][:, j], v, atol=1e-10)
            assert A[n][np.argmax(np.abs(A[n][:, j])), j] > 0


def test_thosvd_exact_for_low_multilinear_rank():
    P = synth.coupled_problem([(6, 7, 5)], 3, (0, 0, 0), None, 4, dtype=np.float64)
    G, A, _ = tucker.thosvd(P.tensors[0], (3, 3, 3))
    np.testing.assert_allclose(brute_tucker(G, A), P.tensors[0], atol=1e-12)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_tucker_identities_match_element_sums(n):
    rng = np.random.default_rng(6)
    G = rng.standard_normal((3, 2, 4))
    A = [np.linalg.qr(rng.standard_normal((d, j)))[0] for d, j in ((5, 3), (4, 2), (6, 4))]
    U = [rng.random((a.shape[0], 3)) for a in A]
    data = TuckerData([G], [A])
    Xt = brute_tucker(G, A)
    np.testing.assert_allclose(data.mttkrp(0, U, n), brute_mttkrp(Xt, U, n), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(data.core_term(0, U), brute_core_term(Xt, U), rtol=1e-12)
    np.testing.assert_allclose(data.dense(0), Xt, atol=1e-12)


def test_kruskal_special_case_is_papers_lra_identity():
    # G = super-diagonal ones, A_n = U~^(n): the Tucker form must give exactly
    # U~^(n) (U~^T U)^{⊛-n} (eq. eqlrau) and (U^T U~)^⊛ 1 (eq. eqlrag)
    rng = np.random.default_rng(8)
    Rt, R = 3, 2
    Ut = [rng.standard_normal((d, Rt)) for d in (5, 4, 6)]
    U = [rng.random((d, R)) for d in (5, 4, 6)]
    G = np.zeros((Rt, Rt, Rt))
    for r in range(Rt):
        G[r, r, r] = 1.0
    data = TuckerData([G], [Ut])
    for n in range(3):
        C = np.ones((Rt, R))
        for m in range(3):
            if m != n:
                C = C * (Ut[m].T @ U[m])
        np.testing.assert_allclose(data.mttkrp(0, U, n), Ut[n] @ C, rtol=1e-12, atol=1e-13)
    C = np.ones((R, Rt))
    for m in range(3):
        C = C * (U[m].T @ Ut[m])
    np.testing.assert_allclose(data.core_term(0, U), C @ np.ones(Rt), rtol=1e-12)


def test_lra_trajectory_equals_dense_when_compression_is_exact():
    # noiseless rank-R blocks have multilinear rank <= R <= J: T-HOSVD is exact
    P = synth.coupled_problem([(8, 7, 6)] * 3, 3, (2, 0, 0), None, 14, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, 3, P.L, 15)
    cores, bases, _ = tucker.compress_all(P.tensors, (4, 4, 4))
    opt = Options(L=P.L)
    a = apg.run(DenseData(P.tensors), U0, lam0, opt, iters=25)
    b = apg.run(TuckerData(cores, bases), U0, lam0, opt, iters=25)
    assert b.restarts == a.restarts
    for s in range(3):
        np.testing.assert_allclose(b.lam[s], a.lam[s], rtol=1e-8)
        for n in range(3):
            np.testing.assert_allclose(b.U[n][s], a.U[n][s], rtol=1e-8, atol=1e-10)


def test_lra_error_triangle_inequality():
    # Proposition 1 (ii), triangle step: ||M - M^|| <= ||M - X~|| + ||X~ - M^||
    P = synth.coupled_problem([(9, 8, 7)] * 2, 3, (3, 0, 0), 10.0, 16, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, 3, P.L, 17)
    cores, bases, _ = tucker.compress_all(P.tensors, (4, 4, 4))
    data = TuckerData(cores, bases)
    st = apg.run(data, U0, lam0, Options(L=P.L), iters=40)
    for s in range(2):
        Mh = apg.reconstruct(st.lam[s], [st.U[n][s] for n in range(3)])
        lhs = np.linalg.norm(P.tensors[s] - Mh)
        rhs = np.linalg.norm(P.tensors[s] - data.dense(s)) + np.linalg.norm(data.dense(s) - Mh)
        assert lhs <= rhs * (1 + 1e-12)
