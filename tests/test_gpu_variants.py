"""Variants of the method described beside the main algorithm, through the C
ABI against the FP64 oracle:

* -NC, core tensors removed (Section III-C): D^(s) is never updated.  With
  the seeded initialisation the cores are merged into the factors (lambda = 1).
* Uneven ranks R^(s) per block (the model of Section II-C): the library embeds
  block s at the common R with zero columns and lambda_r = 0; the oracle runs
  every block at its own rank, without padding.
* Flexible coupling (Section III-C): a mode's shared columns tied only across
  a listed group of blocks; the others keep every column individual (and may
  differ in that mode's size).

Tolerances as in the main parity tests: 1e-5 normwise for FP32 operands,
1e-10 for FP64 (1e-8 for factors after a 50-iteration FP64 trajectory).
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


def make_model(P, U0, lam0, dev, compute, R=None, **kw):
    import torch
    from paper_2302_05119_amd import CoupledCP
    tens = [torch.from_numpy(np.ascontiguousarray(X)).to(dev) for X in P.tensors]
    return CoupledCP(tens, R or P.R, P.L, compute=compute, init_U=U0, init_lambda=lam0, **kw)


def rounded(st, to32):
    st = copy.deepcopy(st)
    if to32:
        st.U = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U]
        st.U_prev = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U_prev]
    return st


def forced_step(dev, P, U0, lam0, compute, k_before, opt, R, **kw):
    """Oracle for k_before iterations, the state loaded into the library, then
    one iteration on both sides."""
    data = DenseData(P.tensors)
    st = apg.run(data, U0, lam0, opt, iters=k_before)
    st = rounded(st, compute != "f64")
    st.F = apg.objective(data, st.lam, st.U)
    st.relerr = apg.relerr(data, st.lam, st.U)
    m = make_model(P, st.U, st.lam, dev, compute, R=R, **kw)
    Lu_prev = [[st.Lu_prev[n][s] for n in range(3)] for s in range(P.S)]
    m.set_state(st.U, st.lam, st.U_prev, st.lam_prev, st.Ld_prev, Lu_prev, st.LC_prev, t=st.t, k=st.k)
    new = apg.iterate(data, st, opt)
    s1 = m.step(1)
    return m, st, new, s1


# ---------------------------------------------------------------------------
# -NC
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("f64", 1e-10)])
def test_nc_one_iteration_teacher_forced(dev, compute, tol):
    say(f"[nc] teacher-forced compute={compute}")
    dtype = np.float64 if compute == "f64" else np.float32
    L = (3, 0, 2)
    P = synth.coupled_problem([(17, 70, 40), (17, 45, 40)], 6, L, 10.0, 211, dtype=dtype)
    U0, lam0 = synth.uniform_init(P.dims, 6, L, 212)
    m, st, new, s1 = forced_step(dev, P, U0, lam0, compute, 3, Options(L=L, update_core=False), 6,
                                 update_core=False)
    say(f"   F gpu={s1['F']:.12e} oracle={new.F:.12e}")
    assert bool(s1["restarted_last"]) == bool(new.last_restarted)
    assert abs(s1["F"] - new.F) / new.F <= tol
    for s in range(P.S):
        np.testing.assert_array_equal(m.lam(s), st.lam[s])
        for n in range(3):
            e = rel(m.factor(n, s), new.U[n][s])
            assert e <= tol, (n, s, e)


def test_nc_fp64_trajectory(dev):
    # 2 blocks of 30^3, R = 5, mode 1 shared, 20 dB; -NC for 50 iterations
    say("[nc] fp64 trajectory")
    name = "c1_fp64_2x30cube_r5"
    P = synth.make_workload(name)
    U0, lam0 = synth.workload_init(name, P)
    m = make_model(P, U0, lam0, dev, "f64", update_core=False)
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=P.L, update_core=False), iters=50)
    s = m.step(50)
    say(f"   F gpu={s['F']:.15e} oracle={ref.F:.15e} restarts gpu={s['restarts']} oracle={ref.restarts}")
    assert s["restarts"] == ref.restarts
    assert abs(s["F"] - ref.F) / ref.F <= 1e-10
    for b in range(2):
        np.testing.assert_array_equal(m.lam(b), lam0[b])
        for n in range(3):
            assert rel(m.factor(n, b), ref.U[n][b]) <= 1e-8


def test_nc_seeded_init_merges_core_into_factors(dev):
    import torch
    from paper_2302_05119_amd import CoupledCP
    say("[nc] seeded init")
    P = synth.coupled_problem([(20, 21, 22)] * 2, 4, (4, 0, 0), 5.0, 221)
    tens = [torch.from_numpy(X).to(dev) for X in P.tensors]
    m = CoupledCP(tens, 4, (4, 0, 0), seed=9, update_core=False)
    for s in range(2):
        np.testing.assert_array_equal(m.lam(s), np.ones(4))
    m.step(10)
    for s in range(2):
        np.testing.assert_array_equal(m.lam(s), np.ones(4))
    ref = CoupledCP(tens, 4, (4, 0, 0), seed=9)
    np.testing.assert_array_equal(ref.factor(1, 1), CoupledCP(tens, 4, (4, 0, 0), seed=9, update_core=False).factor(1, 1))


# ---------------------------------------------------------------------------
# uneven R^(s)
# ---------------------------------------------------------------------------

def uneven_init(P, R, L, ranks, seed):
    U0, lam0 = synth.uniform_init(P.dims, R, L, seed)
    U = [[u[:, :ranks[s]].copy() for s, u in enumerate(per)] for per in U0]
    return U, [l[:ranks[s]].copy() for s, l in enumerate(lam0)]


def check_padding_zero(m, ranks):
    for s, r in enumerate(ranks):
        assert np.all(m.lam(s, padded=True)[r:] == 0.0)
        for n in range(3):
            assert np.all(m.factor(n, s, padded=True)[:, r:] == 0.0)


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("f64", 1e-10)])
@pytest.mark.parametrize("k_before", [0, 3])
def test_uneven_ranks_one_iteration_teacher_forced(dev, compute, tol, k_before):
    say(f"[uneven] teacher-forced compute={compute} k_before={k_before}")
    dtype = np.float64 if compute == "f64" else np.float32
    L, ranks = (3, 0, 2), (6, 3, 5)
    P = synth.coupled_problem([(17, 70, 40), (17, 45, 40), (17, 33, 40)], 6, L, 10.0, 231, dtype=dtype)
    U0, lam0 = uneven_init(P, 6, L, ranks, 232)
    m, st, new, s1 = forced_step(dev, P, U0, lam0, compute, k_before, Options(L=L), 6, block_ranks=ranks)
    say(f"   F gpu={s1['F']:.12e} oracle={new.F:.12e}")
    assert bool(s1["restarted_last"]) == bool(new.last_restarted)
    assert abs(s1["F"] - new.F) / new.F <= tol
    Ld, Lu, LC = m.lipschitz()
    ltol = 1e-6 if compute == "f32" else 1e-11
    np.testing.assert_allclose(Ld, new.Ld_prev, rtol=ltol)
    np.testing.assert_allclose(LC, new.LC_prev, rtol=ltol)
    for s in range(P.S):
        np.testing.assert_allclose(Lu[s], [new.Lu_prev[n][s] for n in range(3)], rtol=ltol)
        assert m.lam(s).shape == (ranks[s],)
        assert rel(m.lam(s), new.lam[s]) <= tol
        for n in range(3):
            assert m.factor(n, s).shape == (P.dims[s][n], ranks[s])
            e = rel(m.factor(n, s), new.U[n][s])
            assert e <= tol, (n, s, e)
    check_padding_zero(m, ranks)


def test_uneven_ranks_fp64_trajectory(dev):
    say("[uneven] fp64 trajectory")
    L, ranks = (2, 0, 0), (5, 2, 4, 3)
    P = synth.coupled_problem([(20, 24, 18), (20, 16, 30), (20, 24, 18), (20, 9, 12)], 5, L, 15.0, 241,
                              dtype=np.float64)
    U0, lam0 = uneven_init(P, 5, L, ranks, 242)
    m = make_model(P, U0, lam0, dev, "f64", R=5, block_ranks=ranks)
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=L), iters=40)
    s = m.step(40)
    say(f"   F gpu={s['F']:.15e} oracle={ref.F:.15e} restarts gpu={s['restarts']} oracle={ref.restarts}")
    assert s["restarts"] == ref.restarts
    assert abs(s["F"] - ref.F) / ref.F <= 1e-10
    for b in range(4):
        assert rel(m.lam(b), ref.lam[b]) <= 1e-8
        for n in range(3):
            assert rel(m.factor(n, b), ref.U[n][b]) <= 1e-8
    check_padding_zero(m, ranks)
    assert m.global_fit() == pytest.approx(apg.fit(P.tensors, ref.lam, ref.U), abs=1e-10)


def test_uneven_ranks_padding_input_is_ignored(dev):
    # the stride-R arrays' columns past R^(s) are ignored on input
    say("[uneven] padding input ignored")
    L, ranks = (2, 0, 0), (4, 2)
    P = synth.coupled_problem([(12, 14, 16)] * 2, 4, L, 20.0, 251, dtype=np.float64)
    U0, lam0 = synth.uniform_init(P.dims, 4, L, 252)
    a = make_model(P, U0, lam0, dev, "f64", block_ranks=ranks)
    Ut, lt = uneven_init(P, 4, L, ranks, 252)
    b = make_model(P, Ut, lt, dev, "f64", block_ranks=ranks)
    check_padding_zero(a, ranks)
    sa, sb = a.step(5), b.step(5)
    assert sa["F"] == sb["F"]
    for s in range(2):
        np.testing.assert_array_equal(a.lam(s), b.lam(s))
        for n in range(3):
            np.testing.assert_array_equal(a.factor(n, s), b.factor(n, s))


# ---------------------------------------------------------------------------
# flexible coupling (Section III-C): coupling on specific blocks only
# ---------------------------------------------------------------------------

GROUPS = ((0, 2, 3), None, (1, 2))      # mode 1: blocks 0, 2, 3; mode 3: blocks 1, 2


def group_init(P, R, L, groups, seed):
    """U[0,1] start whose shared columns agree inside each group only."""
    rng = np.random.default_rng(seed)
    U = [[rng.random((d[n], R)) for d in P.dims] for n in range(3)]
    for n in range(3):
        if L[n]:
            grp = range(P.S) if groups[n] is None else sorted(groups[n])
            grp = list(grp)
            for s in grp[1:]:
                U[n][s][:, :L[n]] = U[n][grp[0]][:, :L[n]]
    lam = [rng.random(R) for _ in range(P.S)]
    return U, lam


def group_problem(dtype):
    # block 1 is outside mode 1's group, so its I_1 may differ
    dims = [(17, 40, 30), (11, 45, 30), (17, 33, 30), (17, 40, 26)]
    return synth.coupled_problem(dims, 6, (0, 0, 0), 10.0, 261, dtype=dtype)


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("f64", 1e-10)])
@pytest.mark.parametrize("k_before", [0, 3])
def test_flexible_coupling_one_iteration_teacher_forced(dev, compute, tol, k_before):
    say(f"[flex] teacher-forced compute={compute} k_before={k_before}")
    dtype = np.float64 if compute == "f64" else np.float32
    L = (3, 0, 2)
    P = group_problem(dtype)
    P.L = L
    U0, lam0 = group_init(P, 6, L, GROUPS, 262)
    opt = Options(L=L, coupled_blocks=GROUPS)
    m, st, new, s1 = forced_step(dev, P, U0, lam0, compute, k_before, opt, 6, coupled_blocks=GROUPS)
    say(f"   F gpu={s1['F']:.12e} oracle={new.F:.12e}")
    assert bool(s1["restarted_last"]) == bool(new.last_restarted)
    assert abs(s1["F"] - new.F) / new.F <= tol
    Ld, Lu, LC = m.lipschitz()
    ltol = 1e-6 if compute == "f32" else 1e-11
    np.testing.assert_allclose(LC, new.LC_prev, rtol=ltol)
    for s in range(P.S):
        np.testing.assert_allclose(Lu[s], [new.Lu_prev[n][s] for n in range(3)], rtol=ltol)
        assert rel(m.lam(s), new.lam[s]) <= tol
        for n in range(3):
            e = rel(m.factor(n, s), new.U[n][s])
            assert e <= tol, (n, s, e)
    # members share their columns bit for bit; the others are free
    for n, grp in ((0, GROUPS[0]), (2, GROUPS[2])):
        ref = m.factor(n, grp[0])[:, :L[n]]
        for s in grp[1:]:
            np.testing.assert_array_equal(m.factor(n, s)[:, :L[n]], ref)
    assert not np.array_equal(m.factor(2, 0)[:, :2], m.factor(2, 1)[:, :2])


def test_flexible_coupling_fp64_trajectory(dev):
    say("[flex] fp64 trajectory")
    L = (3, 0, 2)
    P = group_problem(np.float64)
    P.L = L
    U0, lam0 = group_init(P, 6, L, GROUPS, 272)
    m = make_model(P, U0, lam0, dev, "f64", R=6, coupled_blocks=GROUPS)
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=L, coupled_blocks=GROUPS), iters=40)
    s = m.step(40)
    say(f"   F gpu={s['F']:.15e} oracle={ref.F:.15e} restarts gpu={s['restarts']} oracle={ref.restarts}")
    assert s["restarts"] == ref.restarts
    assert abs(s["F"] - ref.F) / ref.F <= 1e-10
    for b in range(P.S):
        assert rel(m.lam(b), ref.lam[b]) <= 1e-8
        for n in range(3):
            assert rel(m.factor(n, b), ref.U[n][b]) <= 1e-8


def test_flexible_coupling_seeded_init_and_rejections(dev):
    import torch
    from paper_2302_05119_amd import ConcpdError, CoupledCP
    say("[flex] seeded init, rejections")
    P = group_problem(np.float32)
    tens = [torch.from_numpy(X).to(dev) for X in P.tensors]
    m = CoupledCP(tens, 6, (3, 0, 2), seed=4, coupled_blocks=GROUPS)
    for n, grp in ((0, GROUPS[0]), (2, GROUPS[2])):
        L = (3, 0, 2)[n]
        for s in grp[1:]:
            np.testing.assert_array_equal(m.factor(n, s)[:, :L], m.factor(n, grp[0])[:, :L])
    assert not np.array_equal(m.factor(2, 0)[:, :2], m.factor(2, 1)[:, :2])   # block 0 is outside mode 3's group
    with pytest.raises(ConcpdError):
        CoupledCP(tens, 6, (3, 0, 0))                               # block 1's I_1 differs
    with pytest.raises(ConcpdError):
        CoupledCP(tens, 6, (3, 0, 0), coupled_blocks=((), None, None))  # empty group
    with pytest.raises(ConcpdError):
        CoupledCP(tens, 6, (3, 0, 0), coupled_blocks=((0, 1), None, None))  # unequal I_1 inside the group


def test_variants_together_on_the_lra_path(dev):
    # -NC, uneven ranks and flexible coupling at once, on T-HOSVD compressed
    # blocks (Algorithm 2): 30 iterations against the oracle on its own
    # compression (fit of X~ and global fit at 1e-4)
    from oracle import tucker
    from oracle.apg import TuckerData
    say("[variants] lra: -NC + uneven ranks + coupling groups")
    L, ranks, J = (3, 0, 2), (6, 4, 5, 6), (8, 8, 8)
    P = group_problem(np.float32)
    P.L = L
    U6, lam6 = group_init(P, 6, L, GROUPS, 282)
    U0 = [[U6[n][s][:, :ranks[s]].copy() for s in range(P.S)] for n in range(3)]
    lam0 = [lam6[s][:ranks[s]].copy() for s in range(P.S)]
    cores, bases, _ = tucker.compress_all([X.astype(np.float64) for X in P.tensors], J)
    opt = Options(L=L, coupled_blocks=GROUPS, update_core=False)
    ref = apg.run(TuckerData(cores, bases), U0, lam0, opt, iters=30)
    m = make_model(P, U0, lam0, dev, "f32", R=6, block_ranks=ranks, coupled_blocks=GROUPS, update_core=False,
                   tucker_ranks=J)
    m.lra_compress()
    s = m.lra_step(30)
    gf = m.global_fit()
    rf = apg.fit(P.tensors, ref.lam, ref.U)
    say(f"   fit(X~) gpu={s['fit']:.8f} oracle={1 - ref.relerr:.8f}; global gpu={gf:.8f} oracle={rf:.8f}")
    assert s["k"] == 30
    assert abs(s["fit"] - (1 - ref.relerr)) <= 1e-4
    assert abs(gf - rf) <= 1e-4
    for b in range(P.S):
        np.testing.assert_array_equal(m.lam(b), lam0[b])
    check_padding_zero(m, ranks)
    for n, grp in ((0, GROUPS[0]), (2, GROUPS[2])):
        for b in grp[1:]:
            np.testing.assert_array_equal(m.factor(n, b)[:, :L[n]], m.factor(n, grp[0])[:, :L[n]])
