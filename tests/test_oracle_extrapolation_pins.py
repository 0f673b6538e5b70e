"""Pins of the oracle's extrapolated sweep, its weights, RelErr and the stopping
rule, against values this file computes without the oracle's formulas:

* one accepted extrapolated sweep (eq. eqextraPG / eqextraPU with the weights
  of eq. eqextrawd / eqextrawu and the shared-block weight of the joint update,
  eq. solUnC) is rebuilt block by block from the objective alone: every
  gradient is a central finite difference of the element-sum objective at the
  extrapolated point, every Lipschitz constant the largest eigenvalue of a
  second-difference Hessian of that objective, and w_hat comes from the decimal
  values of t_k and w_hat_{k-1} = (t_{k-1} - 1) / t_k (Appendix A, parameter
  settings), not from the recursion;
* RelErr (Section III-C, termination criteria) against an element-sum
  reconstruction;
* the stopping rule (Section III-C: stop once |RelErr_k - RelErr_{k-1}| < tol, or
  at MaxIt) against a RelErr history computed here.

The objective is quadratic in every block, so central differences are exact up
to rounding and the comparisons can be tight.
"""
import numpy as np
import pytest

from oracle import apg
from oracle.apg import DenseData, Options
import synth
import test_oracle_pins as pins

# t_k, k = 0..7, and w_hat_{k-1} = (t_{k-1} - 1) / t_k, k = 1..7, to ten decimals
T_TABLE = [1.0, 1.6180339887, 2.1935270853, 2.7497913401, 3.2948796779, 3.8326014001,
           4.3650787175, 4.8936217645]
W_TABLE = [0.0, 0.2817535251, 0.4340427828, 0.5310638054, 0.5987785941, 0.6489233261, 0.6876458540]
DELTA_W = 0.9999


def _fd_grad(f, x, h=1e-3):
    g = np.zeros_like(x)
    for idx in np.ndindex(x.shape):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        g[idx] = (f(xp) - f(xm)) / (2.0 * h)
    return g


def _fd_hessian(f, x, h=0.25):
    n = x.size
    H = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            def at(sa, sb):
                y = x.copy().ravel()
                y[a] += sa * h
                y[b] += sb * h
                return f(y.reshape(x.shape))
            H[a, b] = (at(1, 1) - at(1, -1) - at(-1, 1) + at(-1, -1)) / (4.0 * h * h)
    return 0.5 * (H + H.T)


def _lmax(H):
    return float(np.linalg.eigvalsh(H)[-1])


def _weight(w_hat, L_prev, L_cur):
    return min(w_hat, DELTA_W * np.sqrt(L_prev / L_cur))


def _copyU(U):
    return [[u.copy() for u in per] for per in U]


def expected_extrapolated_sweep(tensors, st, w_hat, L, groups):
    """One extrapolated sweep in the Gauss-Seidel order (cores, then modes
    1..3), every number taken from element-sum evaluations of F."""
    S, N = len(st.lam), 3
    U = _copyU(st.U)
    lam = [l.copy() for l in st.lam]
    F = lambda lm, Uu: pins.brute_F(tensors, lm, Uu)  # noqa: E731

    for s in range(S):
        def f_lam(x, s=s):
            lm = [l.copy() for l in lam]
            lm[s] = x
            return F(lm, U)
        Ld = _lmax(_fd_hessian(f_lam, lam[s]))
        w = _weight(w_hat, st.Ld_prev[s], Ld)
        lam_hat = st.lam[s] + w * (st.lam[s] - st.lam_prev[s])
        g = _fd_grad(f_lam, lam_hat)
        lam[s] = np.maximum(0.0, lam_hat - g / Ld)

    for n in range(N):
        Ln = L[n]
        grp = ([] if Ln == 0 else list(range(S)) if groups is None or groups[n] is None
               else sorted(groups[n]))
        Lu = []
        for s in range(S):
            def f_row(x, s=s):
                Uu = _copyU(U)
                Uu[n][s] = Uu[n][s].copy()
                Uu[n][s][0, :] = x
                return F(lam, Uu)
            Lu.append(_lmax(_fd_hessian(f_row, U[n][s][0, :].copy())))
        Uhat = []
        for s in range(S):
            w = _weight(w_hat, st.Lu_prev[n][s], Lu[s])
            Uhat.append(st.U[n][s] + w * (st.U[n][s] - st.U_prev[n][s]))
        if grp:
            LC = sum(Lu[s] for s in grp)
            wC = _weight(w_hat, st.LC_prev[n], LC)
            g0 = grp[0]
            UC_hat = st.U[n][g0][:, :Ln] + wC * (st.U[n][g0][:, :Ln] - st.U_prev[n][g0][:, :Ln])
            for s in grp:
                Uhat[s][:, :Ln] = UC_hat
        Uat = _copyU(U)
        for s in range(S):
            Uat[n][s] = Uhat[s].copy()
        new = [None] * S
        if grp:
            def f_shared(x):
                Uu = _copyU(Uat)
                for s in grp:
                    Uu[n][s][:, :Ln] = x
                return F(lam, Uu)
            gC = _fd_grad(f_shared, UC_hat.copy())
            UC_new = np.maximum(0.0, UC_hat - gC / LC)
        for s in range(S):
            Ls = Ln if s in grp else 0

            def f_ind(x, s=s, Ls=Ls):
                Uu = _copyU(Uat)
                Uu[n][s][:, Ls:] = x
                return F(lam, Uu)
            gI = _fd_grad(f_ind, Uhat[s][:, Ls:].copy())
            UI_new = np.maximum(0.0, Uhat[s][:, Ls:] - gI / Lu[s])
            new[s] = np.concatenate([UC_new, UI_new], axis=1) if Ls else UI_new
        for s in range(S):
            U[n][s] = new[s]
    return lam, U


CASES = {
    # every weight equals w_hat (the Lipschitz-ratio cap cannot bind)
    "cap_free": dict(dims=((3, 4, 2), (3, 5, 2)), L=(1, 0, 1), groups=None, prev=(1e30, 1e30, 1e30)),
    # the cap binds everywhere, with different previous constants for the cores,
    # the individual blocks and the shared blocks
    "cap_binds": dict(dims=((3, 4, 2), (3, 5, 2)), L=(1, 0, 1), groups=None, prev=(2e-4, 5e-4, 1e-4)),
    # a coupling group in mode 1 (blocks 0 and 2), cap binding
    "group": dict(dims=((3, 4, 2), (3, 3, 2), (3, 4, 2)), L=(1, 0, 0), groups=((0, 2), None, None),
                  prev=(3e-4, 6e-4, 1e-4)),
}


@pytest.mark.parametrize("k", [2, 4, 7])
@pytest.mark.parametrize("case", sorted(CASES))
def test_extrapolated_sweep_from_objective_evaluations(case, k):
    c = CASES[case]
    R = 2
    P = synth.coupled_problem(list(c["dims"]), R, c["L"], 10.0, 61, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, R, c["L"], 62)
    S = len(P.dims)
    data = DenseData(P.tensors)
    opt = Options(L=c["L"], coupled_blocks=c["groups"])
    st = apg.initial_state(data, U0, lam0)
    rng = np.random.default_rng(63)
    # x_{k-2}: a perturbed copy of x_{k-1}, shared columns still tied within groups
    st.U_prev = [[u * (1.0 + 0.6 * (rng.random(u.shape) - 0.5)) for u in per] for per in st.U]
    for n in range(3):
        if c["L"][n]:
            grp = list(range(S)) if c["groups"] is None or c["groups"][n] is None else sorted(c["groups"][n])
            for s in grp[1:]:
                st.U_prev[n][s][:, :c["L"][n]] = st.U_prev[n][grp[0]][:, :c["L"][n]]
    st.lam_prev = [l * (1.0 + 0.6 * (rng.random(l.shape) - 0.5)) for l in st.lam]
    pd, pu, pc = c["prev"]
    st.Ld_prev = [pd] * S
    st.Lu_prev = [[pu * (1 + 0.1 * s) for s in range(S)] for _ in range(3)]
    st.LC_prev = [pc] * 3
    st.t = T_TABLE[k - 1]
    st.F = np.inf          # accept the extrapolated sweep
    new = apg.iterate(data, st, opt)
    assert not new.last_restarted
    assert new.t == pytest.approx(T_TABLE[k], rel=1e-10)
    lam_e, U_e = expected_extrapolated_sweep(P.tensors, st, W_TABLE[k - 1], c["L"], c["groups"])
    for s in range(S):
        np.testing.assert_allclose(new.lam[s], lam_e[s], rtol=1e-7, atol=1e-9)
        for n in range(3):
            np.testing.assert_allclose(new.U[n][s], U_e[n][s], rtol=1e-7, atol=1e-9)


# ---------------------------------------------------------------------------
# RelErr and the stopping rule (Section III-C, termination criteria)
# ---------------------------------------------------------------------------

def brute_relerr(tensors, lam, U):
    vals = []
    for s, X in enumerate(tensors):
        Xh = pins.brute_reconstruct(lam[s], [U[n][s] for n in range(3)])
        vals.append(np.sqrt(np.sum((X - Xh) ** 2)) / np.sqrt(np.sum(X * X)))
    return float(np.mean(vals))


def test_relerr_and_fit_match_element_sum_reconstruction():
    P, U0, lam0 = pins.small_problem(dims=((4, 5, 3), (4, 6, 3), (4, 3, 3)), R=3, L=(2, 0, 1), snr=5.0, seed=71)
    data = DenseData(P.tensors)
    st = apg.run(data, U0, lam0, Options(L=P.L), iters=6)
    for lam, U in ((lam0, U0), (st.lam, st.U)):
        ref = brute_relerr(P.tensors, lam, U)
        assert apg.relerr(data, lam, U) == pytest.approx(ref, rel=1e-12)
        assert apg.fit(P.tensors, lam, U) == pytest.approx(1.0 - ref, rel=1e-12)
    assert st.relerr == pytest.approx(brute_relerr(P.tensors, st.lam, st.U), rel=1e-12)


def _history(data, tensors, U0, lam0, opt, kmax):
    st = apg.initial_state(data, U0, lam0)
    hist = [brute_relerr(tensors, st.lam, st.U)]
    states = [st]
    for _ in range(kmax):
        st = apg.iterate(data, st, opt)
        states.append(st)
        hist.append(brute_relerr(tensors, st.lam, st.U))
    return hist, states


@pytest.mark.parametrize("tol", [1e-3, 1e-4])
def test_run_stops_at_first_small_relerr_change_and_at_max_it(tol):
    P, U0, lam0 = pins.small_problem(dims=((4, 5, 3), (4, 6, 3)), R=3, L=(2, 0, 1), snr=10.0, seed=73)
    data = DenseData(P.tensors)
    opt = Options(L=P.L, tol=tol, max_it=300)
    hist, states = _history(data, P.tensors, U0, lam0, opt, 300)
    d = np.abs(np.diff(hist))
    k_stop = int(np.argmax(d < tol)) + 1
    assert d[k_stop - 1] < tol and k_stop >= 3
    # the decision is not a rounding tie
    assert d[k_stop - 1] < tol * (1 - 1e-6) and np.all(d[:k_stop - 1] > tol * (1 + 1e-6))
    r = apg.run(data, U0, lam0, opt)
    assert r.k == k_stop
    assert r.relerr == pytest.approx(hist[k_stop], rel=1e-12)
    for n in range(3):
        for s in range(2):
            np.testing.assert_array_equal(r.U[n][s], states[k_stop].U[n][s])
    # MaxIt caps the run before the rule fires
    capped = apg.run(data, U0, lam0, Options(L=P.L, tol=tol, max_it=k_stop - 2))
    assert capped.k == k_stop - 2
    # tol = 0 never fires: exactly MaxIt iterations
    assert apg.run(data, U0, lam0, Options(L=P.L, tol=0.0, max_it=7)).k == 7
    # a fixed iteration count ignores the rule
    assert apg.run(data, U0, lam0, opt, iters=k_stop + 3).k == k_stop + 3
