"""Order N > 3 (the N-way model of Section II-C, eq. tensormodel) through the
C ABI against the FP64 oracle, which is written for any order.

* MTTKRP of every mode (the dimension-tree passes and contractions the sweep
  uses) on ragged shapes: several 64-row output groups with a partial last
  one, contraction parts with a short last chunk, rows of odd length (scalar
  loads) and of a multiple of 16 bytes (vector loads), R with padded and
  exact 4-column tiles; tolerance 1e-5 (FP32) / 1e-12 (FP64) of max |K|.
* One teacher-forced iteration at N = 4 and 5 with coupled modes: state from
  the oracle after k iterations (FP32-rounded factors for the FP32 path),
  one step on both sides; F, lambda, factors within 1e-5 / 1e-10, Lipschitz
  constants within 1e-6 / 1e-11 (the tolerances of the order-3 tests).
* FP64 trajectories at N = 4 and 6 and an FP32 one at N = 4 (final fit).
* Entry points that exist at order 3 only return ENOTSUP.
"""
import copy
import sys

import numpy as np
import pytest

import synth
from oracle import apg
from oracle.apg import DenseData, Options

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    return torch.device("cuda:0")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(a - b)
    n = np.linalg.norm(b)
    return d / n if n > 0 else d


def make_model(P, U0, lam0, dev, compute, **kw):
    import torch
    from paper_2302_05119_amd import CoupledCP
    tens = [torch.from_numpy(np.ascontiguousarray(X)).to(dev) for X in P.tensors]
    return CoupledCP(tens, P.R, P.L, compute=compute, init_U=U0, init_lambda=lam0, **kw)


MTTKRP_CASES = [
    # dims per block, R, compute
    ([(7, 9, 11, 13), (5, 9, 6, 20)], 6, "f32"),      # odd rows (scalar loads), two block shapes
    ([(20, 30, 40, 50)], 10, "f32"),                  # A = 600, B = 2000: many parts, vector loads
    ([(3, 70, 5, 33)], 16, "f32"),                    # exact 4-column tiles, ragged output groups
    ([(2, 3, 500, 9)], 5, "f32"),                     # lopsided: the split puts three modes first
    ([(4, 5, 6, 7, 3)], 4, "f32"),                    # N = 5
    ([(3, 4, 3, 5, 4, 3)], 3, "f32"),                 # N = 6
    ([(6, 5, 7, 9), (6, 8, 7, 4)], 5, "f64"),
    ([(9, 10, 11, 12, 5)], 7, "f64"),                 # N = 5
    ([(4, 40, 3, 66)], 40, "f32"),                    # R = 40
]


@pytest.mark.parametrize("dims,R,compute", MTTKRP_CASES)
def test_nway_mttkrp_matches_oracle(dev, dims, R, compute):
    say(f"[nway mttkrp] dims={dims} R={R} compute={compute}")
    dtype = np.float64 if compute == "f64" else np.float32
    N = len(dims[0])
    P = synth.coupled_problem(dims, R, (0,) * N, 10.0, 501, dtype=dtype)
    U0, lam0 = synth.uniform_init(P.dims, R, (0,) * N, 502)
    m = make_model(P, U0, lam0, dev, compute)
    tol = 1e-12 if compute == "f64" else 1e-5
    for s in range(P.S):
        Us = [m.factor(n, s) for n in range(N)]
        X = P.tensors[s].astype(np.float64)
        for n in range(N):
            Kg = m.debug_mttkrp(n, s).cpu().numpy()
            Kr = apg.mttkrp(X, Us, n)
            e = np.max(np.abs(Kg - Kr)) / np.max(np.abs(Kr))
            say(f"   s={s} n={n} max-rel={e:.2e}")
            assert e <= tol


def _teacher_forced(dev, P, R, L, compute, k_before, seed):
    N = len(L)
    U0, lam0 = synth.uniform_init(P.dims, R, L, seed)
    data = DenseData(P.tensors)
    opt = Options(L=L)
    st = apg.run(data, U0, lam0, opt, iters=k_before)
    st = copy.deepcopy(st)
    if compute != "f64":
        st.U = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U]
        st.U_prev = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U_prev]
    st.F = apg.objective(data, st.lam, st.U)
    st.relerr = apg.relerr(data, st.lam, st.U)
    m = make_model(P, st.U, st.lam, dev, compute)
    Lu_prev = [[st.Lu_prev[n][s] for n in range(N)] for s in range(P.S)]
    m.set_state(st.U, st.lam, st.U_prev, st.lam_prev, st.Ld_prev, Lu_prev, st.LC_prev, t=st.t, k=st.k)
    s0 = m.stats()
    new = apg.iterate(data, st, opt)
    s1 = m.step(1)
    return m, st, new, s0, s1


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("f64", 1e-10)])
@pytest.mark.parametrize("k_before", [0, 3])
@pytest.mark.parametrize("order", [4, 5])
def test_nway_one_iteration_teacher_forced(dev, compute, tol, k_before, order):
    say(f"[nway step] N={order} compute={compute} k_before={k_before}")
    dtype = np.float64 if compute == "f64" else np.float32
    if order == 4:
        L = (3, 0, 2, 0)
        dims = [(11, 14, 9, 17), (11, 10, 9, 17), (11, 14, 9, 12)]
    else:
        L = (2, 0, 0, 1, 0)
        dims = [(6, 7, 5, 8, 9), (6, 4, 5, 8, 7)]
    P = synth.coupled_problem(dims, 6, L, 10.0, 601 + order, dtype=dtype)
    m, st, new, s0, s1 = _teacher_forced(dev, P, 6, L, compute, k_before, 602 + order)
    say(f"   F_prev gpu={s0['F']:.12e} oracle={st.F:.12e}; F gpu={s1['F']:.12e} oracle={new.F:.12e} "
        f"restart gpu={s1['restarted_last']} oracle={new.last_restarted}")
    assert abs(s0["F"] - st.F) / st.F <= tol
    assert bool(s1["restarted_last"]) == bool(new.last_restarted)
    assert abs(s1["F"] - new.F) / new.F <= tol
    Ld, Lu, LC = m.lipschitz()
    ltol = 1e-6 if compute == "f32" else 1e-11
    np.testing.assert_allclose(Ld, new.Ld_prev, rtol=ltol)
    np.testing.assert_allclose(LC, new.LC_prev, rtol=ltol)
    for s in range(P.S):
        np.testing.assert_allclose(Lu[s], [new.Lu_prev[n][s] for n in range(order)], rtol=ltol)
        assert rel(m.lam(s), new.lam[s]) <= tol
        for n in range(order):
            e = rel(m.factor(n, s), new.U[n][s])
            assert e <= tol, (n, s, e)
            # elementwise, relative to the factor's largest entry
            d = np.max(np.abs(m.factor(n, s) - new.U[n][s])) / np.max(np.abs(new.U[n][s]))
            assert d <= 2 * tol, (n, s, d)
    # the shared columns stay identical across the blocks
    for n in range(order):
        if L[n]:
            for s in range(1, P.S):
                np.testing.assert_array_equal(m.factor(n, s)[:, :L[n]], m.factor(n, 0)[:, :L[n]])


@pytest.mark.parametrize("dims,L,iters", [
    ([(8, 9, 10, 11)] * 2, (4, 0, 0, 2), 30),
    ([(4, 5, 3, 4, 5, 3)] * 2, (0, 2, 0, 0, 0, 0), 20),
])
def test_nway_fp64_trajectory_matches_oracle(dev, dims, L, iters):
    N = len(L)
    say(f"[nway trajectory] N={N} dims={dims} L={L} iters={iters}")
    P = synth.coupled_problem(dims, 5, L, 20.0, 701 + N, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, 5, L, 702 + N)
    m = make_model(P, U0, lam0, dev, "f64")
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=L), iters=iters)
    s = m.step(iters)
    say(f"   F gpu={s['F']:.15e} oracle={ref.F:.15e} restarts gpu={s['restarts']} oracle={ref.restarts}")
    assert s["k"] == iters and s["restarts"] == ref.restarts
    assert abs(s["F"] - ref.F) / ref.F <= 1e-10
    for b in range(P.S):
        assert rel(m.lam(b), ref.lam[b]) <= 1e-8
        for n in range(N):
            assert rel(m.factor(n, b), ref.U[n][b]) <= 1e-8
    gf = m.global_fit()
    assert gf == pytest.approx(apg.fit(P.tensors, ref.lam, ref.U), abs=1e-10)


def test_nway_fp32_run_to_stop_final_fit(dev):
    # N = 4, three blocks, stopping rule of Section III-C on both sides
    L = (3, 0, 0, 3)
    P = synth.coupled_problem([(12, 15, 10, 14)] * 3, 5, L, 20.0, 801, dtype=np.float32)
    U0, lam0 = synth.uniform_init(P.dims, 5, L, 802)
    U32 = [[u.astype(np.float32).astype(np.float64) for u in per] for per in U0]
    ref = apg.run(DenseData(P.tensors), U32, lam0, Options(L=L, tol=1e-8, max_it=400))
    m = make_model(P, U0, lam0, dev, "f32", tol=1e-8, max_it=400)
    st = m.fit()
    gf = m.global_fit()
    rf = apg.fit(P.tensors, ref.lam, ref.U)
    say(f"[nway fp32 to stop] k gpu={st['k']} oracle={ref.k}; fit gpu={gf:.8f} oracle={rf:.8f}")
    assert 1 <= st["k"] <= 400 and st["converged"] == int(st["k"] < 400)
    assert abs(gf - rf) <= 1e-3
    assert gf > 0.8


def test_nway_graph_sweeps_match_direct(dev):
    L = (2, 0, 0, 0)
    P = synth.coupled_problem([(9, 8, 7, 10)] * 2, 4, L, 15.0, 901, dtype=np.float32)
    U0, lam0 = synth.uniform_init(P.dims, 4, L, 902)
    a = make_model(P, U0, lam0, dev, "f32")
    b = make_model(P, U0, lam0, dev, "f32")
    b.set_option("graph_sweeps", 4)
    sa, sb = a.step(12), b.step(12)
    assert sa["F"] == sb["F"] and sa["k"] == sb["k"] == 12
    for n in range(4):
        for s in range(2):
            np.testing.assert_array_equal(a.factor(n, s), b.factor(n, s))


def test_nway_state_round_trip(dev):
    L = (2, 0, 0, 0)
    P = synth.coupled_problem([(9, 8, 7, 10)] * 2, 4, L, 15.0, 903, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, 4, L, 904)
    a = make_model(P, U0, lam0, dev, "f64")
    a.step(5)
    state = a.get_state()
    assert len(state["U"]) == 4 and len(state["Lu_prev"][0]) == 4 and len(state["LC_prev"]) == 4
    b = make_model(P, U0, lam0, dev, "f64")
    b.set_state(**state)
    sa, sb = a.step(4), b.step(4)
    assert sa["F"] == sb["F"]
    for n in range(4):
        np.testing.assert_array_equal(a.factor(n, 1), b.factor(n, 1))


def test_nway_order3_only_entry_points_return_enotsup(dev):
    from paper_2302_05119_amd._lib import ConcpdError
    P = synth.coupled_problem([(6, 7, 8, 9)], 3, (0, 0, 0, 0), 10.0, 905, dtype=np.float32)
    U0, lam0 = synth.uniform_init(P.dims, 3, (0, 0, 0, 0), 906)
    m = make_model(P, U0, lam0, dev, "f32")
    calls = [lambda: m.lra_compress_cp(), lambda: m.autotune(2), lambda: m.set_option("fuse", 0),
             lambda: m.profile(True)]
    for call in calls:
        with pytest.raises(ConcpdError) as ei:
            call()
        assert ei.value.status == 2, str(ei.value)
    # the context keeps working afterwards
    assert m.step(2)["k"] == 2
