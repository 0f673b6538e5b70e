"""Pins of the FP64 oracle at tensor order N > 3 (the N-way model of
Section II-C): the MTTKRP, the core data term, the reconstruction and the
objective against plain element loops; the Hadamard-of-Grams identity of
Appendix A against an explicit Khatri-Rao Gram; gradients against central
finite differences of F; the descent and restart properties of Algorithm 1;
exact recovery of a noiseless coupled 4-way model."""
import itertools

import numpy as np
import pytest

from oracle import apg
from oracle.apg import DenseData, Options
import synth


def brute_mttkrp(X, U, n):
    R = U[0].shape[1]
    K = np.zeros((X.shape[n], R))
    for idx in itertools.product(*[range(d) for d in X.shape]):
        for r in range(R):
            p = X[idx]
            for m in range(X.ndim):
                if m != n:
                    p *= U[m][idx[m], r]
            K[idx[n], r] += p
    return K


def brute_model(lam, U, idx):
    v = 0.0
    for r in range(len(lam)):
        p = lam[r]
        for m in range(len(U)):
            p *= U[m][idx[m], r]
        v += p
    return v


def brute_F(tensors, lam, U):
    tot = 0.0
    for s, X in enumerate(tensors):
        Us = [U[m][s] for m in range(X.ndim)]
        for idx in itertools.product(*[range(d) for d in X.shape]):
            tot += 0.5 * (X[idx] - brute_model(lam[s], Us, idx)) ** 2
    return tot


def problem4(dims=((3, 4, 2, 3), (3, 2, 2, 4)), R=3, L=(2, 0, 1, 0), snr=20.0, seed=11):
    P = synth.coupled_problem(list(dims), R, L, snr, seed, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, R, L, seed + 100)
    return P, U0, lam0


@pytest.mark.parametrize("shape", [(3, 4, 2, 3), (2, 3, 2, 2, 3)])
def test_nway_mttkrp_matches_element_sum(shape):
    rng = np.random.default_rng(12)
    X = rng.standard_normal(shape)
    U = [rng.random((d, 3)) for d in shape]
    for n in range(len(shape)):
        np.testing.assert_allclose(apg.mttkrp(X, U, n), brute_mttkrp(X, U, n), rtol=1e-13, atol=1e-13)


def test_nway_core_term_reconstruction_objective_match_element_sums():
    rng = np.random.default_rng(13)
    shape = (2, 3, 4, 2)
    X = rng.standard_normal(shape)
    U = [rng.random((d, 2)) for d in shape]
    lam = rng.random(2)
    b = np.zeros(2)
    for idx in itertools.product(*[range(d) for d in shape]):
        for r in range(2):
            b[r] += X[idx] * np.prod([U[m][idx[m], r] for m in range(4)])
    np.testing.assert_allclose(apg.core_data_term(X, U), b, rtol=1e-13)
    Xh = apg.reconstruct(lam, U)
    for idx in itertools.product(*[range(d) for d in shape]):
        assert Xh[idx] == pytest.approx(brute_model(lam, U, idx), rel=1e-13, abs=1e-15)
    P, U0, lam0 = problem4()
    assert apg.objective(DenseData(P.tensors), lam0, U0) == pytest.approx(brute_F(P.tensors, lam0, U0), rel=1e-13)


def test_nway_hadamard_of_grams_equals_explicit_krp_gram():
    rng = np.random.default_rng(14)
    U = [rng.random((d, 3)) for d in (2, 3, 2, 3)]
    rows = [U[0][a] * U[1][b] * U[2][c] * U[3][d]
            for a, b, c, d in itertools.product(range(2), range(3), range(2), range(3))]
    KR = np.array(rows)
    np.testing.assert_allclose(apg.hadamard_of_grams(U), KR.T @ KR, rtol=1e-13)
    rows = [U[0][a] * U[1][b] * U[3][d] for a, b, d in itertools.product(range(2), range(3), range(3))]
    KR = np.array(rows)
    np.testing.assert_allclose(apg.hadamard_of_grams(U, skip=2), KR.T @ KR, rtol=1e-13)


def test_nway_gradients_match_finite_differences():
    P, U0, lam0 = problem4()
    data = DenseData(P.tensors)
    F, g_lam, g_U, g_C = apg.loss_and_grads(data, lam0, U0, P.L)
    h = 1e-6

    def Fat(lam, U):
        return apg.objective(data, lam, U)

    for s in range(2):
        for r in range(3):
            lp = [l.copy() for l in lam0]
            lm = [l.copy() for l in lam0]
            lp[s][r] += h
            lm[s][r] -= h
            assert (Fat(lp, U0) - Fat(lm, U0)) / (2 * h) == pytest.approx(g_lam[s][r], rel=1e-6, abs=1e-7)
    for n in range(4):
        for s in range(2):
            for (i, r) in [(0, 0), (P.dims[s][n] - 1, 2)]:
                Up = [[u.copy() for u in per] for per in U0]
                Um = [[u.copy() for u in per] for per in U0]
                Up[n][s][i, r] += h
                Um[n][s][i, r] -= h
                fd = (Fat(lam0, Up) - Fat(lam0, Um)) / (2 * h)
                assert fd == pytest.approx(g_U[n][s][i, r], rel=1e-6, abs=1e-7)
    # a shared column is one parameter of every block: its gradient is the sum over s
    for n in (0, 2):
        for r in range(P.L[n]):
            for i in range(P.dims[0][n]):
                Up = [[u.copy() for u in per] for per in U0]
                Um = [[u.copy() for u in per] for per in U0]
                for s in range(2):
                    Up[n][s][i, r] += h
                    Um[n][s][i, r] -= h
                fd = (Fat(lam0, Up) - Fat(lam0, Um)) / (2 * h)
                assert fd == pytest.approx(g_C[n][i, r], rel=1e-6, abs=1e-7)


def test_nway_unextrapolated_sweep_never_increases_objective():
    P, U0, lam0 = problem4(dims=((3, 4, 2, 3), (3, 4, 2, 3)), L=(2, 2, 1, 0), snr=0.0, seed=15)
    data = DenseData(P.tensors)
    st = apg.initial_state(data, U0, lam0)
    for _ in range(8):
        lam, U, _ = apg.sweep(data, st, 0.0, False, Options(L=P.L))
        F = apg.objective(data, lam, U)
        assert F <= st.F * (1 + 1e-14)
        for n in range(4):
            for s in range(2):
                assert np.all(U[n][s] >= 0.0)
                if P.L[n]:
                    np.testing.assert_array_equal(U[n][s][:, :P.L[n]], U[n][0][:, :P.L[n]])
        st = apg.State(U=U, lam=lam, U_prev=st.U, lam_prev=st.lam, Ld_prev=st.Ld_prev,
                       Lu_prev=st.Lu_prev, LC_prev=st.LC_prev, F=F)


def test_nway_forced_overshoot_triggers_restart():
    P, U0, lam0 = problem4()
    data = DenseData(P.tensors)
    opt = Options(L=P.L)
    st = apg.run(data, U0, lam0, opt, iters=4)
    st.U_prev = [[u - 50.0 for u in per] for per in st.U]
    st.lam_prev = [l - 50.0 for l in st.lam]
    st.t = 50.0
    new = apg.iterate(data, st, opt)
    assert new.last_restarted and new.F <= st.F


def test_nway_noiseless_exact_rank_recovery():
    P = synth.coupled_problem([(6, 5, 4, 5)] * 2, 2, (2, 0, 0, 0), None, 16, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, 2, P.L, 17)
    st = apg.run(DenseData(P.tensors), U0, lam0, Options(L=P.L, tol=0.0), iters=1500)
    assert 1 - st.relerr >= 0.999
