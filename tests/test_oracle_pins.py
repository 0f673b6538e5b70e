"""Pins of the FP64 oracle against facts it does not itself compute:
brute-force element sums, finite differences, exact block minimisers,
closed forms and invariants of the method."""
import itertools

import numpy as np
import pytest

from oracle import apg
from oracle.apg import DenseData, Options
import synth


# ---------------------------------------------------------------------------
# independent brute-force helpers (plain loops over tensor elements)
# ---------------------------------------------------------------------------

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


def brute_core_term(X, U):
    R = U[0].shape[1]
    b = np.zeros(R)
    for idx in itertools.product(*[range(d) for d in X.shape]):
        for r in range(R):
            p = X[idx]
            for m in range(X.ndim):
                p *= U[m][idx[m], r]
            b[r] += p
    return b


def brute_reconstruct(lam, U):
    shape = [u.shape[0] for u in U]
    X = np.zeros(shape)
    for idx in itertools.product(*[range(d) for d in shape]):
        v = 0.0
        for r in range(len(lam)):
            p = lam[r]
            for m in range(len(U)):
                p *= U[m][idx[m], r]
            v += p
        X[idx] = v
    return X


def brute_F(tensors, lam, U):
    tot = 0.0
    for s, X in enumerate(tensors):
        for idx in itertools.product(*[range(d) for d in X.shape]):
            v = 0.0
            for r in range(len(lam[s])):
                p = lam[s][r]
                for m in range(3):
                    p *= U[m][s][idx[m], r]
                v += p
            tot += 0.5 * (X[idx] - v) ** 2
    return tot


def small_problem(dims=((4, 5, 3), (4, 6, 3)), R=3, L=(2, 0, 1), snr=20.0, seed=7):
    P = synth.coupled_problem(list(dims), R, L, snr, seed, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, R, L, seed + 100)
    return P, U0, lam0


# ---------------------------------------------------------------------------
# P1: MTTKRP / core data term / reconstruction against element sums
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [0, 1, 2])
def test_mttkrp_matches_element_sum(n):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4, 5, 3))
    U = [rng.random((d, 3)) for d in X.shape]
    np.testing.assert_allclose(apg.mttkrp(X, U, n), brute_mttkrp(X, U, n), rtol=1e-13, atol=1e-13)


def test_core_term_and_reconstruction_match_element_sums():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((3, 4, 5))
    U = [rng.random((d, 2)) for d in X.shape]
    lam = rng.random(2)
    np.testing.assert_allclose(apg.core_data_term(X, U), brute_core_term(X, U), rtol=1e-13)
    np.testing.assert_allclose(apg.reconstruct(lam, U), brute_reconstruct(lam, U), rtol=1e-13, atol=1e-14)


def test_objective_matches_element_sum():
    P, U0, lam0 = small_problem()
    F = apg.objective(DenseData(P.tensors), lam0, U0)
    assert F == pytest.approx(brute_F(P.tensors, lam0, U0), rel=1e-13)


def test_unfold_fold_roundtrip_and_kolda_index():
    X = np.arange(24.0).reshape(2, 3, 4)
    X1 = apg.unfold(X, 1)
    # Kolda: column j = i1 + I1 * i3 for mode 2 (0-based: modes 0 and 2 remain)
    for i1, i2, i3 in itertools.product(range(2), range(3), range(4)):
        assert X1[i2, i1 + 2 * i3] == X[i1, i2, i3]
    for n in range(3):
        np.testing.assert_array_equal(apg.fold(apg.unfold(X, n), n, X.shape), X)


# ---------------------------------------------------------------------------
# P2: Hadamard-of-Grams identity (Appendix A: (U^⊙)^T U^⊙ = (U^T U)^⊛)
# ---------------------------------------------------------------------------

def test_hadamard_of_grams_equals_explicit_krp_gram():
    rng = np.random.default_rng(5)
    U = [rng.random((d, 4)) for d in (3, 5, 2)]
    # explicit KRP built by loops, independent of apg.khatri_rao
    rows = []
    for i3, i2, i1 in itertools.product(range(2), range(5), range(3)):
        rows.append(U[0][i1] * U[1][i2] * U[2][i3])
    KR = np.array(rows)
    np.testing.assert_allclose(apg.hadamard_of_grams(U), KR.T @ KR, rtol=1e-13)
    rows = [U[0][i1] * U[2][i3] for i3, i1 in itertools.product(range(2), range(3))]
    KR = np.array(rows)
    np.testing.assert_allclose(apg.hadamard_of_grams(U, skip=1), KR.T @ KR, rtol=1e-13)


# ---------------------------------------------------------------------------
# P3 / P4: gradients by central finite differences of F
# ---------------------------------------------------------------------------

def test_gradients_match_finite_differences():
    P, U0, lam0 = small_problem()
    data = DenseData(P.tensors)
    L = P.L
    F, g_lam, g_U, g_C = apg.loss_and_grads(data, lam0, U0, L)
    h = 1e-6

    def Fat(lam, U):
        return apg.objective(data, lam, U)

    for s in range(2):
        for r in range(3):
            lp = [l.copy() for l in lam0]
            lm = [l.copy() for l in lam0]
            lp[s][r] += h
            lm[s][r] -= h
            fd = (Fat(lp, U0) - Fat(lm, U0)) / (2 * h)
            assert fd == pytest.approx(g_lam[s][r], rel=1e-6, abs=1e-7)
    for n in range(3):
        for s in range(2):
            for (i, r) in [(0, 0), (1, 2), (P.dims[s][n] - 1, 1)]:
                Up = [[u.copy() for u in per] for per in U0]
                Um = [[u.copy() for u in per] for per in U0]
                Up[n][s][i, r] += h
                Um[n][s][i, r] -= h
                fd = (Fat(lam0, Up) - Fat(lam0, Um)) / (2 * h)
                assert fd == pytest.approx(g_U[n][s][i, r], rel=1e-6, abs=1e-7)
    # shared column: one parameter used by every block -> gradient is the sum over s
    for n in range(3):
        for r in range(L[n]):
            for i in range(P.dims[0][n]):
                Up = [[u.copy() for u in per] for per in U0]
                Um = [[u.copy() for u in per] for per in U0]
                for s in range(2):
                    Up[n][s][i, r] += h
                    Um[n][s][i, r] -= h
                fd = (Fat(lam0, Up) - Fat(lam0, Um)) / (2 * h)
                assert fd == pytest.approx(g_C[n][i, r], rel=1e-6, abs=1e-7)


# ---------------------------------------------------------------------------
# P5: Lipschitz constants
# ---------------------------------------------------------------------------

def power_iteration(A, iters=5000):
    x = np.ones(A.shape[0])
    for _ in range(iters):
        y = A @ x
        x = y / np.linalg.norm(y)
    return float(x @ A @ x)


def test_spectral_norm_is_block_lipschitz_constant():
    P, U0, lam0 = small_problem()
    data = DenseData(P.tensors)
    s, n = 1, 1
    Us = [U0[m][s] for m in range(3)]
    Pm = np.outer(lam0[s], lam0[s]) * apg.hadamard_of_grams(Us, skip=n)
    L = apg.spectral_norm(Pm)
    assert L == pytest.approx(power_iteration(Pm), rel=1e-10)
    assert L == pytest.approx(np.linalg.norm(Pm, 2), rel=1e-12)

    # ||grad(U + d) - grad(U)|| <= L ||d||, with equality along the top eigvector
    def grad_block(Ublock):
        U = [[u.copy() for u in per] for per in U0]
        U[n][s] = Ublock
        return apg.loss_and_grads(data, lam0, U, (0, 0, 0))[2][n][s]

    g0 = grad_block(U0[n][s])
    rng = np.random.default_rng(1)
    for _ in range(5):
        d = rng.standard_normal(U0[n][s].shape)
        ratio = np.linalg.norm(grad_block(U0[n][s] + d) - g0) / np.linalg.norm(d)
        assert ratio <= L * (1 + 1e-12)
    v = np.linalg.eigh(Pm)[1][:, -1]
    d = np.zeros_like(U0[n][s])
    d[0] = v
    ratio = np.linalg.norm(grad_block(U0[n][s] + d) - g0) / np.linalg.norm(d)
    assert ratio == pytest.approx(L, rel=1e-9)


# ---------------------------------------------------------------------------
# P6: t_k recursion (Appendix A)
# ---------------------------------------------------------------------------

def test_t_sequence_closed_forms():
    t = [1.0]
    for _ in range(50):
        t.append(apg.t_next(t[-1]))
    assert t[1] == pytest.approx((1 + 5 ** 0.5) / 2, rel=1e-15)
    for k in range(1, 51):
        # t_k solves t^2 - t - t_{k-1}^2 = 0 and grows at least like (k+2)/2
        assert t[k] ** 2 - t[k] == pytest.approx(t[k - 1] ** 2, rel=1e-13)
        assert t[k] >= (k + 2) / 2 - 1e-12
        assert t[k] <= k + 1
    w = [(t[k - 1] - 1) / t[k] for k in range(1, 51)]
    assert w[0] == 0.0
    assert all(0 <= a < b < 1 for a, b in zip(w[1:], w[2:]))


def test_extrapolation_weight_rule():
    assert apg.extrapolation_weight(0.5, None, 3.0, 0.9999) == 0.0
    assert apg.extrapolation_weight(0.5, 4.0, 1.0, 0.9999) == 0.5
    assert apg.extrapolation_weight(0.9, 1.0, 4.0, 0.9999) == pytest.approx(0.9999 * 0.5)
    assert apg.extrapolation_weight(0.5, 1.0, 0.0, 0.9999) == 0.0


# ---------------------------------------------------------------------------
# Exact block minimiser (R = 1): every block's Hessian is a multiple of I, so an
# unextrapolated prox-gradient step with step 1/L is the exact nonnegative
# minimiser of F over that block.  Compute the minimiser coordinate-wise from
# three evaluations of F alone and compare with the oracle's sweep.
# ---------------------------------------------------------------------------

def _coord_min(Ffun, x0):
    """argmin_{x >= 0} of a 1-D quadratic sampled at x0-1, x0, x0+1."""
    fm, f0, fp = Ffun(x0 - 1.0), Ffun(x0), Ffun(x0 + 1.0)
    a = 0.5 * (fp + fm - 2 * f0)
    b = 0.5 * (fp - fm)
    return max(0.0, x0 - b / (2 * a))


@pytest.mark.parametrize("update_core", [True, False])
@pytest.mark.parametrize("L,groups", [((0, 0, 0), None), ((1, 0, 1), None), ((1, 1, 1), None),
                                      ((1, 0, 1), ((0, 2), None, (1, 2))), ((1, 1, 0), ((1,), (0, 1, 2), None))])
def test_unextrapolated_sweep_is_exact_block_minimisation_rank1(L, groups, update_core):
    # update_core=False is the -NC variant (Section III-C, no core update): the lambda
    # coordinates are skipped and only the factor blocks are minimised.  groups:
    # flexible coupling (Section III-C), the shared coordinate is tied only
    # across the listed blocks of that mode.
    P = synth.coupled_problem([(3, 4, 2), (3, 4, 2), (3, 4, 2)], 1, L, 10.0, 11, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, 1, L, 12)
    opt = Options(L=L, update_core=update_core, coupled_blocks=groups)
    S = 3

    def group_of(n):
        if not L[n]:
            return []
        return list(range(S)) if groups is None or groups[n] is None else sorted(groups[n])

    for n in range(3):
        # the start ties the shared column only inside the group
        grp = group_of(n)
        for s in range(S):
            if L[n] and s not in grp:
                U0[n][s] = U0[n][s] * (1.0 + 0.3 * (s + 1))
    data = DenseData(P.tensors)
    st = apg.initial_state(data, U0, lam0)
    lam_new, U_new, _ = apg.sweep(data, st, 0.0, False, opt)

    lam = [l.copy() for l in lam0]
    U = [[u.copy() for u in per] for per in U0]
    F = lambda lm, Uu: apg.objective(data, lm, Uu)  # noqa: E731
    for s in range(S if update_core else 0):
        def fl(x, s=s):
            lm = [l.copy() for l in lam]
            lm[s][0] = x
            return F(lm, U)
        lam[s][0] = _coord_min(fl, lam[s][0])
    for n in range(3):
        newU = [u.copy() for u in U[n]]
        grp = group_of(n)
        if L[n] == 1:
            # shared column: one coordinate per row, set in every group block at once
            for i in range(P.dims[0][n]):
                def fc(x, i=i):
                    Uu = [[u.copy() for u in per] for per in U]
                    for s in grp:
                        Uu[n][s][i, 0] = x
                    return F(lam, Uu)
                v = _coord_min(fc, U[n][grp[0]][i, 0])
                for s in grp:
                    newU[s][i, 0] = v
        for s in range(S):
            if L[n] == 1 and s in grp:
                continue
            for i in range(P.dims[s][n]):
                def fi(x, i=i, s=s):
                    Uu = [[u.copy() for u in per] for per in U]
                    Uu[n][s][i, 0] = x
                    return F(lam, Uu)
                newU[s][i, 0] = _coord_min(fi, U[n][s][i, 0])
        U[n] = newU
    for s in range(S):
        np.testing.assert_allclose(lam_new[s], lam[s], rtol=1e-9)
        for n in range(3):
            np.testing.assert_allclose(U_new[n][s], U[n][s], rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------------------
# P7 / P8 / P9: whole-algorithm invariants
# ---------------------------------------------------------------------------

def test_restart_keeps_objective_monotone_and_factors_nonnegative():
    P, U0, lam0 = small_problem(dims=((5, 6, 4), (5, 7, 4), (5, 6, 4)), R=3, L=(2, 0, 1), snr=10.0)
    data = DenseData(P.tensors)
    opt = Options(L=P.L)
    st = apg.initial_state(data, U0, lam0)
    F_prev = st.F
    for _ in range(60):
        st = apg.iterate(data, st, opt)
        assert st.F <= F_prev * (1 + 1e-14)
        F_prev = st.F
        for n in range(3):
            for s in range(3):
                assert np.all(st.U[n][s] >= 0)
                if P.L[n]:
                    np.testing.assert_array_equal(st.U[n][s][:, :P.L[n]], st.U[n][0][:, :P.L[n]])
        assert all(np.all(l >= 0) for l in st.lam)


def test_nc_variant_keeps_core_and_stays_monotone():
    # -NC (Section III-C): D^(s) never changes, bit for bit, and the accepted
    # objective still never increases, with restarts on.
    P, U0, lam0 = small_problem(dims=((5, 6, 4), (5, 7, 4)), R=3, L=(2, 0, 1), snr=10.0, seed=23)
    data = DenseData(P.tensors)
    opt = Options(L=P.L, update_core=False)
    st = apg.initial_state(data, U0, lam0)
    F_prev = st.F
    for _ in range(40):
        st = apg.iterate(data, st, opt)
        assert st.F <= F_prev * (1 + 1e-14)
        F_prev = st.F
        for s in range(2):
            np.testing.assert_array_equal(st.lam[s], lam0[s])
    full = apg.run(data, U0, lam0, Options(L=P.L), iters=40)
    assert not np.allclose(full.lam[0], lam0[0])


def test_unextrapolated_sweep_never_increases_objective():
    P, U0, lam0 = small_problem(dims=((4, 5, 3), (4, 5, 3)), R=4, L=(2, 2, 2), snr=0.0, seed=21)
    data = DenseData(P.tensors)
    st = apg.initial_state(data, U0, lam0)
    for _ in range(10):
        lam, U, _ = apg.sweep(data, st, 0.0, False, Options(L=P.L))
        F = apg.objective(data, lam, U)
        assert F <= st.F * (1 + 1e-14)
        st = apg.State(U=U, lam=lam, U_prev=st.U, lam_prev=st.lam, Ld_prev=st.Ld_prev,
                       Lu_prev=st.Lu_prev, LC_prev=st.LC_prev, F=F)


def test_forced_overshoot_triggers_restart():
    P, U0, lam0 = small_problem(snr=20.0)
    data = DenseData(P.tensors)
    opt = Options(L=P.L)
    st = apg.run(data, U0, lam0, opt, iters=5)
    # make x_{k-2} far from x_{k-1} so that the extrapolated point overshoots
    st.U_prev = [[u - 50.0 for u in per] for per in st.U]
    st.lam_prev = [l - 50.0 for l in st.lam]
    st.t = 50.0
    new = apg.iterate(data, st, opt)
    assert new.last_restarted
    assert new.F <= st.F


def test_noiseless_exact_rank_recovery():
    P = synth.coupled_problem([(12, 11, 10)] * 2, 3, (3, 0, 0), None, 31, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, 3, P.L, 32)
    data = DenseData(P.tensors)
    st = apg.run(data, U0, lam0, Options(L=P.L, tol=0.0), iters=1500)
    assert 1 - st.relerr >= 0.9999


def test_kkt_complementarity_at_convergence():
    P = synth.coupled_problem([(8, 7, 6)] * 2, 3, (2, 0, 0), 15.0, 41, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, 3, P.L, 42)
    data = DenseData(P.tensors)
    st = apg.run(data, U0, lam0, Options(L=P.L, tol=0.0), iters=3000)
    _, g_lam, g_U, g_C = apg.loss_and_grads(data, st.lam, st.U, P.L)
    for n in range(3):
        for s in range(2):
            Ln = P.L[n]
            scale = np.linalg.norm(apg.mttkrp(data.X[s], [st.U[m][s] for m in range(3)], n) * st.lam[s])
            gi = g_U[n][s][:, Ln:]
            assert np.linalg.norm(np.minimum(st.U[n][s][:, Ln:], gi)) / scale < 1e-5
            assert gi.min() / scale > -1e-5
        if P.L[n]:
            scale = np.linalg.norm(g_C[n]) + np.linalg.norm(st.U[n][0][:, :P.L[n]])
            assert np.linalg.norm(np.minimum(st.U[n][0][:, :P.L[n]], g_C[n])) / scale < 1e-5


# ---------------------------------------------------------------------------
# Identities the HIP path relies on, checked with the oracle's primitives
# ---------------------------------------------------------------------------

def test_core_term_reuse_and_objective_expansion():
    P, U0, lam0 = small_problem()
    data = DenseData(P.tensors)
    for s in range(2):
        Us = [U0[n][s] for n in range(3)]
        b = apg.core_data_term(data.X[s], Us)
        for n in range(3):
            K = apg.mttkrp(data.X[s], Us, n)
            np.testing.assert_allclose(np.sum(K * Us[n], axis=0), b, rtol=1e-12)
        H = apg.hadamard_of_grams(Us)
        F_exp = 0.5 * (np.sum(data.X[s] ** 2) - 2 * lam0[s] @ b + lam0[s] @ H @ lam0[s])
        r = data.X[s] - apg.reconstruct(lam0[s], Us)
        assert F_exp == pytest.approx(0.5 * np.sum(r * r), rel=1e-11)


def _uneven(U0, lam0, ranks):
    U = [[u[:, :ranks[s]].copy() for s, u in enumerate(per)] for per in U0]
    return U, [l[:ranks[s]].copy() for s, l in enumerate(lam0)]


def test_uneven_ranks_native_equal_zero_padded():
    # Section II-C lets each block have its own R^(s) (>= every L_n).  The
    # oracle runs the blocks at their own ranks; the padded run embeds them at
    # R = max R^(s) with zero columns and lambda_r = 0, and must agree.
    ranks = (4, 2, 3)
    P, U0, lam0 = small_problem(dims=((5, 6, 4), (5, 7, 4), (5, 8, 4)), R=4, L=(2, 0, 1), snr=10.0, seed=41)
    Un, ln = _uneven(U0, lam0, ranks)
    Up = [[np.concatenate([u, np.zeros((u.shape[0], 4 - u.shape[1]))], axis=1) for u in per] for per in Un]
    lp = [np.concatenate([l, np.zeros(4 - l.size)]) for l in ln]
    data = DenseData(P.tensors)
    a = apg.run(data, Un, ln, Options(L=P.L), iters=8)
    b = apg.run(data, Up, lp, Options(L=P.L), iters=8)
    assert a.restarts == b.restarts
    assert b.F == pytest.approx(a.F, rel=1e-12)
    for s, r in enumerate(ranks):
        np.testing.assert_allclose(b.lam[s][:r], a.lam[s], rtol=1e-11)
        assert np.all(b.lam[s][r:] == 0.0)
        for n in range(3):
            np.testing.assert_allclose(b.U[n][s][:, :r], a.U[n][s], rtol=1e-11, atol=1e-14)
            assert np.all(b.U[n][s][:, r:] == 0.0)
            if P.L[n]:
                np.testing.assert_array_equal(a.U[n][s][:, :P.L[n]], a.U[n][0][:, :P.L[n]])


def test_zero_padding_of_components_is_exact():
    # uneven R by zero columns with lambda_r = 0 (the padded columns stay 0)
    P, U0, lam0 = small_problem(R=3, L=(0, 0, 0))
    Upad = [[np.concatenate([u, np.zeros((u.shape[0], 1))], axis=1) for u in per] for per in U0]
    lpad = [np.concatenate([l, [0.0]]) for l in lam0]
    data = DenseData(P.tensors)
    a = apg.run(data, U0, lam0, Options(L=P.L), iters=5)
    b = apg.run(data, Upad, lpad, Options(L=P.L), iters=5)
    for s in range(2):
        np.testing.assert_allclose(b.lam[s][:3], a.lam[s], rtol=1e-12)
        assert b.lam[s][3] == 0.0
        for n in range(3):
            np.testing.assert_allclose(b.U[n][s][:, :3], a.U[n][s], rtol=1e-12, atol=1e-15)
