"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: relative (normwise) error <= 1e-5 for FP32 factor / gradient
results and <= 1e-10 for the FP64 path; Lipschitz constants are exact
eigenvalues on both sides (FP64), compared at 1e-6 / 1e-11.
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


def elem(a, b):
    """Largest elementwise difference over the largest magnitude: a few wrong
    rows cannot hide under it as they can under a normwise ratio."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m = np.max(np.abs(b)) if b.size else 0.0
    d = np.max(np.abs(a - b)) if b.size else 0.0
    return d / m if m > 0 else d


def make_model(P, U0, lam0, dev, compute, **kw):
    import torch
    from paper_2302_05119_amd import CoupledCP
    tens = [torch.from_numpy(np.ascontiguousarray(X)).to(dev) for X in P.tensors]
    return CoupledCP(tens, P.R, P.L, compute=compute, init_U=U0, init_lambda=lam0, **kw)


def stored_factors(m):
    return [[m.factor(n, s) for s in range(m.S)] for n in range(3)]


MTTKRP_CASES = [
    # dims, R, compute: ragged row groups, chunks, i3 tiles; padded and exact R tiles
    ([(9, 70, 100), (6, 70, 37)], 20, "f32"),
    ([(5, 130, 65)], 7, "f32"),
    ([(13, 20, 200)], 30, "f32"),
    ([(7, 9, 11), (7, 9, 11)], 5, "f64"),
    ([(5, 66, 70)], 12, "f64"),
    # U2 too large for LDS: staged in row chunks (a ragged last chunk)
    ([(3, 700, 40), (6, 300, 20)], 20, "f32"),
    ([(5, 200, 37)], 64, "f32"),
    ([(3, 300, 20)], 32, "f64"),
    # R = 40 (ten 4-column tiles, the 512^3 leg's instantiation), U2 whole
    # and staged in row chunks
    ([(4, 70, 90)], 40, "f32"),
    ([(3, 520, 30)], 40, "f32"),
]


@pytest.mark.parametrize("dims,R,compute", MTTKRP_CASES)
def test_mttkrp_matches_oracle(dev, dims, R, compute):
    say(f"[mttkrp] dims={dims} R={R} compute={compute}")
    dtype = np.float64 if compute == "f64" else np.float32
    P = synth.coupled_problem(dims, R, (0, 0, 0), 10.0, 101, dtype=dtype)
    U0, lam0 = synth.uniform_init(P.dims, R, (0, 0, 0), 102)
    m = make_model(P, U0, lam0, dev, compute)
    tol = 1e-12 if compute == "f64" else 1e-5
    for s in range(P.S):
        Us = [m.factor(n, s) for n in range(3)]
        X = P.tensors[s].astype(np.float64)
        for n in range(3):
            Kg = m.debug_mttkrp(n, s).cpu().numpy()
            Kr = apg.mttkrp(X, Us, n)
            e = np.max(np.abs(Kg - Kr)) / np.max(np.abs(Kr))
            say(f"   s={s} n={n} max-rel={e:.2e}")
            assert e <= tol


def oracle_state_rounded(st, to32):
    st = copy.deepcopy(st)
    if to32:
        st.U = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U]
        st.U_prev = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U_prev]
    return st


def teacher_forced(dev, P, R, L, compute, k_before, seed, overshoot=False, update_core=True):
    U0, lam0 = synth.uniform_init(P.dims, R, L, seed)
    data = DenseData(P.tensors)
    opt = Options(L=L, update_core=update_core)
    st = apg.run(data, U0, lam0, opt, iters=k_before)
    if overshoot:
        st.U_prev = [[u * 0.2 for u in per] for per in st.U]
        st.lam_prev = [l * 0.2 for l in st.lam]
        st.t = 40.0
    st = oracle_state_rounded(st, compute != "f64")
    st.F = apg.objective(data, st.lam, st.U)
    st.relerr = apg.relerr(data, st.lam, st.U)
    m = make_model(P, st.U, st.lam, dev, compute, update_core=update_core)
    Lu_prev = [[st.Lu_prev[n][s] for n in range(3)] for s in range(P.S)]
    m.set_state(st.U, st.lam, st.U_prev, st.lam_prev, st.Ld_prev, Lu_prev, st.LC_prev, t=st.t, k=st.k)
    s0 = m.stats()
    new = apg.iterate(data, st, opt)
    s1 = m.step(1)
    return m, st, new, s0, s1


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("f64", 1e-10)])
@pytest.mark.parametrize("k_before", [0, 4])
def test_one_iteration_teacher_forced(dev, compute, tol, k_before):
    say(f"[step] compute={compute} k_before={k_before}")
    dtype = np.float64 if compute == "f64" else np.float32
    L = (3, 0, 2)
    P = synth.coupled_problem([(17, 70, 40), (17, 45, 40), (17, 70, 40)], 6, L, 10.0, 201, dtype=dtype)
    m, st, new, s0, s1 = teacher_forced(dev, P, 6, L, compute, k_before, 202)
    say(f"   F_prev gpu={s0['F']:.12e} oracle={st.F:.12e}; F gpu={s1['F']:.12e} oracle={new.F:.12e} "
        f"restart gpu={s1['restarted_last']} oracle={new.last_restarted}")
    assert abs(s0["F"] - st.F) / st.F <= tol
    assert bool(s1["restarted_last"]) == bool(new.last_restarted)
    assert abs(s1["F"] - new.F) / new.F <= tol
    Ld, Lu, LC = m.lipschitz()
    ltol = 1e-6 if compute == "f32" else 1e-11
    np.testing.assert_allclose(Ld, new.Ld_prev, rtol=ltol)
    for s in range(P.S):
        np.testing.assert_allclose(Lu[s], [new.Lu_prev[n][s] for n in range(3)], rtol=ltol)
        e = rel(m.lam(s), new.lam[s])
        assert e <= tol, (s, e)
        assert elem(m.lam(s), new.lam[s]) <= tol
        for n in range(3):
            e = rel(m.factor(n, s), new.U[n][s])
            assert e <= tol, (n, s, e)
            # elementwise, relative to the factor's largest entry
            assert elem(m.factor(n, s), new.U[n][s]) <= 2 * tol, (n, s)
    np.testing.assert_allclose(LC, new.LC_prev, rtol=ltol)


def test_restart_path_teacher_forced(dev):
    say("[restart] forced overshoot")
    L = (2, 0, 0)
    P = synth.coupled_problem([(12, 14, 16)] * 2, 4, L, 20.0, 301, dtype=np.float64)
    m, st, new, s0, s1 = teacher_forced(dev, P, 4, L, "f64", 6, 302, overshoot=True)
    assert new.last_restarted and s1["restarted_last"] == 1
    assert s1["restarts"] == 1
    for s in range(2):
        assert rel(m.lam(s), new.lam[s]) <= 1e-10
        for n in range(3):
            assert rel(m.factor(n, s), new.U[n][s]) <= 1e-10


def test_fp64_trajectory_matches_oracle_c1(dev):
    # 2 blocks of 30^3, R = 5, mode-1 factor fully shared, 20 dB, 50 iterations
    say("[c1] fp64 trajectory")
    name = "c1_fp64_2x30cube_r5"
    P = synth.make_workload(name)
    U0, lam0 = synth.workload_init(name, P)
    m = make_model(P, U0, lam0, dev, "f64")
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=P.L), iters=50)
    s = m.step(50)
    say(f"   F gpu={s['F']:.15e} oracle={ref.F:.15e} restarts gpu={s['restarts']} oracle={ref.restarts}")
    assert s["k"] == 50
    assert s["restarts"] == ref.restarts
    assert abs(s["F"] - ref.F) / ref.F <= 1e-10
    for b in range(2):
        assert rel(m.lam(b), ref.lam[b]) <= 1e-8
        for n in range(3):
            assert rel(m.factor(n, b), ref.U[n][b]) <= 1e-8
    gf = m.global_fit()
    assert gf == pytest.approx(apg.fit(P.tensors, ref.lam, ref.U), abs=1e-10)


def test_fp32_trajectory_final_fit(dev):
    say("[fp32] trajectory fit")
    L = (5, 0, 0)
    P = synth.coupled_problem([(40, 36, 50)] * 3, 8, L, 10.0, 401, dtype=np.float32)
    U0, lam0 = synth.uniform_init(P.dims, 8, L, 402)
    m = make_model(P, U0, lam0, dev, "f32")
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=L), iters=40)
    s = m.step(40)
    gf = m.global_fit()
    rf = apg.fit(P.tensors, ref.lam, ref.U)
    say(f"   fit gpu={gf:.8f} oracle={rf:.8f} restarts {s['restarts']} vs {ref.restarts}")
    assert abs(gf - rf) <= 1e-4
    assert abs(s["fit"] - (1 - ref.relerr)) <= 1e-4


def test_full_size_c2_one_iteration_teacher_forced(dev):
    # the benchmark workload: 10 blocks of 100^3, R = 20, 5 shared mode-1 columns
    say("[c2 full] teacher-forced iteration")
    name = "c2_fp32_10x100cube_r20"
    P = synth.make_workload(name)
    w = synth.WORKLOADS[name]
    m, st, new, s0, s1 = teacher_forced(dev, P, w["R"], w["L"], "f32", 1, w["seed"] + 1000)
    say(f"   F gpu={s1['F']:.10e} oracle={new.F:.10e}")
    assert abs(s1["F"] - new.F) / new.F <= 1e-5
    for s in range(P.S):
        assert rel(m.lam(s), new.lam[s]) <= 1e-5
        for n in range(3):
            assert rel(m.factor(n, s), new.U[n][s]) <= 1e-5


def test_seeded_init_and_nonnegativity(dev):
    import torch
    from paper_2302_05119_amd import CoupledCP
    say("[init] seeded init, projection")
    P = synth.coupled_problem([(20, 21, 22)] * 2, 4, (4, 4, 0), 5.0, 501)
    tens = [torch.from_numpy(X).to(dev) for X in P.tensors]
    m = CoupledCP(tens, 4, (4, 4, 0), seed=7)
    m2 = CoupledCP(tens, 4, (4, 4, 0), seed=7)
    for n in range(3):
        for s in range(2):
            np.testing.assert_array_equal(m.factor(n, s), m2.factor(n, s))
    m.step(15)
    for n in range(3):
        for s in range(2):
            U = m.factor(n, s)
            assert np.all(U >= 0)
            if n < 2:
                np.testing.assert_array_equal(U, m.factor(n, 0))
    assert all(np.all(m.lam(s) >= 0) for s in range(2))


@pytest.mark.parametrize("compute", ["f32", "f64"])
def test_checkpoint_get_state_set_state_resumes_bit_for_bit(dev, compute):
    # a checkpoint taken after 7 iterations, restored into a fresh context,
    # continues exactly as the original run (iterate, objective, Lipschitz
    # constants, extrapolation state)
    say(f"[checkpoint] compute={compute}")
    dtype = np.float64 if compute == "f64" else np.float32
    L = (3, 0, 2)
    P = synth.coupled_problem([(17, 40, 30), (17, 25, 30), (17, 33, 30)], 6, L, 10.0, 901, dtype=dtype)
    U0, lam0 = synth.uniform_init(P.dims, 6, L, 902)
    a = make_model(P, U0, lam0, dev, compute)
    a.step(7)
    st = a.get_state()
    assert st["k"] == 7 and st["t"] > 1.0
    for s in range(P.S):
        np.testing.assert_array_equal(st["lam"][s], a.lam(s))
        for n in range(3):
            np.testing.assert_array_equal(st["U"][n][s], a.factor(n, s))
    b = make_model(P, U0, lam0, dev, compute, seed=3)
    b.set_state(**st)
    assert b.stats()["F"] == a.stats()["F"]
    sa, sb = a.step(10), b.step(10)
    say(f"   F a={sa['F']:.15e} b={sb['F']:.15e} k {sa['k']} {sb['k']}")
    assert sa["F"] == sb["F"] and sa["k"] == sb["k"] == 17
    for s in range(P.S):
        np.testing.assert_array_equal(a.lam(s), b.lam(s))
        for n in range(3):
            np.testing.assert_array_equal(a.factor(n, s), b.factor(n, s))
    for x, y in zip(a.lipschitz(), b.lipschitz()):
        np.testing.assert_array_equal(x, y)
