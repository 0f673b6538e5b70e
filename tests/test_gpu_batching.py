"""Batching form: graph replay of sweeps, launch options, the autotuner, and
grouped launches over many blocks of uneven size (EEG-shaped workloads), in
FP32 and in the BF16-operand precision form.

Graph replays are checked bitwise against eager launches of an identical
context after every replay, with eager work and synchronisations between
them.  Precision-form tolerances: FP32 1e-5 per teacher-forced step; BF16
operands 2e-2 per step and final fit within 1e-3 of the FP64 oracle.
"""
import sys

import numpy as np
import pytest

import synth
from paper_2302_05119_amd import ConcpdError
from oracle import apg
from oracle.apg import DenseData, Options

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / n if n > 0 else np.linalg.norm(a - b)


def model(P, U0, lam0, compute="f32", **kw):
    import torch
    from paper_2302_05119_amd import CoupledCP
    dev = torch.device("cuda:0")
    tens = [torch.from_numpy(np.ascontiguousarray(X)).to(dev) for X in P.tensors]
    return CoupledCP(tens, P.R, P.L, compute=compute, init_U=U0, init_lambda=lam0, **kw)


def factors(m):
    return [m.factor(n, s) for n in range(3) for s in range(m.S)]


@pytest.mark.parametrize("gs,overlap", [(1, 0), (4, 0), (1, 1), (4, 1)])
def test_graph_replay_matches_eager(gs, overlap):
    # overlap = 1: the small kernels on the second stream, captured as parallel
    # branches of the graph
    import torch
    say(f"[graph] sweeps per graph = {gs}, overlap = {overlap}")
    L = (2, 0, 0)
    P = synth.coupled_problem([(24, 40, 33), (24, 17, 50), (24, 29, 8)], 6, L, 10.0, 801)
    U0, lam0 = synth.uniform_init(P.dims, 6, L, 802)
    me = model(P, U0, lam0)
    mg = model(P, U0, lam0)
    mg.set_option("overlap", overlap)
    mg.set_option("graph_sweeps", gs)
    assert mg.get_option("graph_sweeps") == gs and mg.get_option("overlap") == overlap
    scratch = torch.zeros(1 << 20, device="cuda:0")
    for rep in range(5):
        se = me.step(gs)
        sg = mg.step(gs)
        # eager work of the program between replays
        scratch.add_(1.0)
        torch.cuda.synchronize()
        assert se["k"] == sg["k"] and se["F"] == sg["F"] and se["restarts"] == sg["restarts"], (rep, se, sg)
        for a, b in zip(factors(me), factors(mg)):
            np.testing.assert_array_equal(a, b)
    # asynchronous replays, then a synchronised check
    me.step(3 * gs, sync=False)
    mg.step(3 * gs, sync=False)
    for a, b in zip(factors(me), factors(mg)):
        np.testing.assert_array_equal(a, b)
    assert float(scratch[0]) == 5.0


def test_k2_rows_option_within_tolerance():
    say("[options] mode-2 chunk rows")
    L = (3, 0, 0)
    P = synth.coupled_problem([(70, 45, 40)] * 3, 8, L, 10.0, 811)
    U0, lam0 = synth.uniform_init(P.dims, 8, L, 812)
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=L), iters=3)
    for k2 in (8, 16, 32, 64):
        m = model(P, U0, lam0)
        m.set_option("k2_rows", k2)
        s = m.step(3)
        e = max(rel(m.factor(n, b), ref.U[n][b]) for n in range(3) for b in range(3))
        say(f"   k2_rows={k2} F={s['F']:.10e} oracle={ref.F:.10e} max factor err={e:.2e}")
        assert abs(s["F"] - ref.F) / ref.F <= 1e-5 and e <= 1e-4


def test_p1_split_option_within_tolerance():
    # 3 x 33 row-group items (a count that needs empty padding items for
    # splits 1 and 2); I3 = 100 spans several 64-byte chunks and a ragged tail
    say("[options] pass-1 split")
    L = (3, 0, 0)
    P = synth.coupled_problem([(33, 45, 100)] * 3, 8, L, 10.0, 815)
    U0, lam0 = synth.uniform_init(P.dims, 8, L, 816)
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=L), iters=3)
    for split in (1, 2, 4, 0):
        m = model(P, U0, lam0)
        m.set_option("p1_split", split)
        assert m.get_option("p1_split") in ((1, 2, 4) if split == 0 else (split,))
        s = m.step(3)
        e = max(rel(m.factor(n, b), ref.U[n][b]) for n in range(3) for b in range(3))
        say(f"   p1_split={split} F={s['F']:.10e} oracle={ref.F:.10e} max factor err={e:.2e}")
        assert abs(s["F"] - ref.F) / ref.F <= 1e-5 and e <= 1e-4
    m = model(P, U0, lam0)
    with pytest.raises(ConcpdError):
        m.set_option("p1_split", 3)


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 2e-2)])
def test_p1_dma_and_register_paths_match_oracle(compute, tol):
    # pass 1 by LDS DMA and through registers, every split, on rows whose
    # last 16-value chunk is ragged (I3 = 100 and 57) and item counts that need
    # empty padding items
    say(f"[options] pass-1 DMA / register paths, compute={compute}")
    L = (3, 0, 0)
    P = synth.coupled_problem([(33, 45, 100), (33, 70, 57), (33, 45, 100)], 8, L, 10.0, 851)
    U0, lam0 = synth.uniform_init(P.dims, 8, L, 852)
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=L), iters=2)
    for dma in (1, 0):
        for split in (1, 2, 4):
            m = model(P, U0, lam0, compute=compute)
            m.set_option("p1_dma", dma)
            m.set_option("p1_split", split)
            assert m.get_option("p1_dma") == dma
            s = m.step(2)
            e = max(rel(m.factor(n, b), ref.U[n][b]) for n in range(3) for b in range(3))
            say(f"   dma={dma} split={split} F={s['F']:.10e} oracle={ref.F:.10e} max factor err={e:.2e}")
            assert abs(s["F"] - ref.F) / ref.F <= tol and e <= 10 * tol


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 2e-2)])
@pytest.mark.parametrize("dims", [[(33, 45, 100), (33, 70, 57), (33, 45, 100)], [(17, 800, 30), (17, 45, 77)]])
def test_pass2_slab_counts_match_oracle(compute, tol, dims, monkeypatch):
    # one or two i1 slabs per pass-2 wavefront (forced at context creation):
    # ragged slab chunks (I1 = 33 and 17 against chunks of 4 and 8 slabs),
    # ragged i3 tiles, and (second case) a U^(2) too long for LDS, which the
    # two-slab kernel restages for each slab
    say(f"[options] pass-2 slabs per wavefront, compute={compute}, dims={dims}")
    L = (3, 0, 0)
    P = synth.coupled_problem(dims, 8, L, 10.0, 861)
    U0, lam0 = synth.uniform_init(P.dims, 8, L, 862)
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=L), iters=2)
    S = len(dims)
    for slabs in ("1", "2"):
        monkeypatch.setenv("CONCPD_P2_SLABS", slabs)
        m = model(P, U0, lam0, compute=compute)
        s = m.step(2)
        e = max(rel(m.factor(n, b), ref.U[n][b]) for n in range(3) for b in range(S))
        say(f"   slabs={slabs} F={s['F']:.10e} oracle={ref.F:.10e} max factor err={e:.2e}")
        assert abs(s["F"] - ref.F) / ref.F <= tol and e <= 10 * tol


def test_profiled_sweeps_leave_the_iterate_unchanged():
    # profiling repeats each MTTKRP pass back to back; the iterate must match
    # an unprofiled twin bit for bit
    say("[profile] repeated pass launches")
    L = (3, 0, 0)
    P = synth.coupled_problem([(40, 45, 60)] * 2, 6, L, 10.0, 841)
    U0, lam0 = synth.uniform_init(P.dims, 6, L, 842)
    a, b = model(P, U0, lam0), model(P, U0, lam0)
    a.step(2)
    b.step(2)
    a.profile(True)
    sa = a.step(3)
    a.profile(False)
    ms1, ms2, n = a.profile_read()
    sb = b.step(3)
    say(f"   pass1 {ms1:.3f} ms pass2 {ms2:.3f} ms over {n} launches")
    assert n >= 12 and n % 4 == 0 and ms1 > 0 and ms2 > 0
    assert sa["k"] == sb["k"] and sa["F"] == sb["F"]
    for x, y in zip(factors(a), factors(b)):
        np.testing.assert_array_equal(x, y)


def test_autotune_keeps_the_iterate():
    say("[autotune]")
    L = (5, 0, 0)
    P = synth.coupled_problem([(60, 60, 60)] * 4, 10, L, 10.0, 821)
    U0, lam0 = synth.uniform_init(P.dims, 10, L, 822)
    m = model(P, U0, lam0)
    m.step(2)
    before, st0 = factors(m), m.stats()
    t = m.autotune(8)
    say(f"   {t}")
    # 60-value FP32 rows are 16-byte aligned: the pass-1 DMA path is a candidate
    assert 18 <= t["candidates"] <= 21 and t["k2_rows"] in (8, 16, 32) and t["graph_sweeps"] in (0, 1, 4)
    assert t["overlap"] in (0, 1) and m.get_option("overlap") == t["overlap"]
    assert t["overlap"] == 0 or t["graph_sweeps"] > 0
    assert t["p1_split"] in (1, 2, 4) and m.get_option("p1_split") == t["p1_split"]
    assert t["p1_dma"] in (0, 1) and m.get_option("p1_dma") == t["p1_dma"]
    assert t["fuse"] in (0, 1) and m.get_option("fuse") == t["fuse"]
    assert t["fuse"] == 0 or t["overlap"] == 0
    assert t["us_per_sweep"] <= t["us_per_sweep_default"]
    st1 = m.stats()
    assert st1["k"] == st0["k"] and st1["F"] == st0["F"]
    for a, b in zip(before, factors(m)):
        np.testing.assert_array_equal(a, b)
    s = m.step(3)
    assert s["k"] == st0["k"] + 3


def eeg_small(seed, S=6, T=(20, 90), R=6):
    return synth.eeg_problem(S, T, R, 5.0, seed, channels=16, freqs=12)


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 2e-2), ("f16", 2e-2)])
def test_uneven_eeg_blocks_teacher_forced(compute, tol):
    say(f"[eeg] uneven blocks, compute={compute}")
    P = eeg_small(831)
    R, L = P.R, P.L
    U0, lam0 = synth.uniform_init(P.dims, R, L, 832)
    data = DenseData(P.tensors)
    opt = Options(L=L)
    st = apg.run(data, U0, lam0, opt, iters=2)
    st.U = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U]
    st.U_prev = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U_prev]
    st.F = apg.objective(data, st.lam, st.U)
    st.relerr = apg.relerr(data, st.lam, st.U)
    m = model(P, st.U, st.lam, compute=compute)
    Lu_prev = [[st.Lu_prev[n][s] for n in range(3)] for s in range(P.S)]
    m.set_state(st.U, st.lam, st.U_prev, st.lam_prev, st.Ld_prev, Lu_prev, st.LC_prev, t=st.t, k=st.k)
    new = apg.iterate(data, st, opt)
    s1 = m.step(1)
    errs = [rel(m.factor(n, b), new.U[n][b]) for n in range(3) for b in range(P.S)]
    errs += [rel(m.lam(b), new.lam[b]) for b in range(P.S)]
    say(f"   F gpu={s1['F']:.10e} oracle={new.F:.10e}; worst factor/lambda error {max(errs):.2e}")
    assert abs(s1["F"] - new.F) / new.F <= tol
    assert max(errs) <= tol


def test_eeg_bf16_final_fit_matches_oracle():
    say("[eeg] BF16 operands, final fit")
    P = synth.eeg_problem(8, (40, 160), 10, 5.0, 841, channels=16, freqs=15)
    U0, lam0 = synth.uniform_init(P.dims, P.R, P.L, 842)
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=P.L), iters=100)
    rf = apg.fit(P.tensors, ref.lam, ref.U)
    for compute in ("bf16", "f16"):
        m = model(P, U0, lam0, compute=compute)
        m.step(100)
        gf = m.global_fit()
        say(f"   {compute}: global fit gpu={gf:.6f} oracle={rf:.6f}")
        assert abs(gf - rf) <= 1e-3


def test_full_size_c4_eeg_teacher_forced_fp32_and_bf16_fit():
    # 16 EEG-shaped blocks 64 x 60 x T_s, T_s in [200, 2000], R = 30, channel
    # and frequency factors fully shared, 5 dB
    name = "c4_eeg_bf16_16blocks_r30"
    say("[c4 full] teacher-forced FP32 and BF16 iteration; BF16 vs FP32 fit")
    P = synth.make_workload(name)
    U0, lam0 = synth.workload_init(name, P)
    U0 = [[u.astype(np.float32).astype(np.float64) for u in per] for per in U0]
    data = DenseData(P.tensors)
    opt = Options(L=P.L)
    new = apg.iterate(data, apg.initial_state(data, U0, lam0), opt)
    m = model(P, U0, lam0, compute="f32")
    s1 = m.step(1)
    say(f"   F gpu={s1['F']:.10e} oracle={new.F:.10e}")
    assert abs(s1["F"] - new.F) / new.F <= 1e-5
    for b in (0, P.S - 1):
        for n in range(3):
            assert rel(m.factor(n, b), new.U[n][b]) <= 1e-5
    m.step(59)
    mb = model(P, U0, lam0, compute="bf16")
    # the BF16 form's first iteration against the same oracle iteration: the
    # per-step bound of the precision form (2e-2), on every block
    sb1 = mb.step(1)
    eb = max(rel(mb.factor(n, b), new.U[n][b]) for b in range(P.S) for n in range(3))
    el = max(rel(mb.lam(b), new.lam[b]) for b in range(P.S))
    say(f"   BF16 step: F gpu={sb1['F']:.10e} oracle={new.F:.10e}; worst factor {eb:.2e}, lambda {el:.2e}")
    assert abs(sb1["F"] - new.F) / new.F <= 2e-2
    assert eb <= 2e-2 and el <= 2e-2
    mb.step(59)
    f32, fb = m.global_fit(), mb.global_fit()
    say(f"   60 iterations: global fit FP32 {f32:.6f}  BF16 {fb:.6f}")
    assert abs(f32 - fb) <= 1e-3


def test_launch_floor_measures_empty_sweeps():
    from paper_2302_05119_amd import launch_floor
    say("[floor] 10 empty kernels")
    f = launch_floor(10, 500)
    say(f"   {f}")
    assert 0.0 < f["graph_us"] < 1e4 and 0.0 < f["direct_us"] < 1e4


@pytest.mark.parametrize("case", ["f32_r20", "f32_r8_groups", "f64_r5", "bf16_dma_r30", "f32_r40_unfused", "f32_uneven_r12"])
def test_fused_launches_bit_identical_to_unfused(case):
    # the R x R work in the launches of the passes it does not depend on:
    # the same arithmetic in the same order, so the iterate must match the
    # unfused sweep bit for bit (restarts and the stopping state included)
    say(f"[fuse] {case}")
    cb = None
    if case == "f32_r20":
        dims, R, L, compute = [(40, 70, 100)] * 3, 20, (5, 0, 0), "f32"
    elif case == "f32_r8_groups":
        dims, R, L, compute = [(30, 45, 60)] * 4, 8, (3, 2, 0), "f32"
        cb = [[0, 2, 3], None, None]
    elif case == "f64_r5":
        dims, R, L, compute = [(30, 30, 30)] * 2, 5, (5, 0, 0), "f64"
    elif case == "bf16_dma_r30":
        dims, R, L, compute = [(33, 45, 64), (33, 70, 57)], 30, (30, 0, 0), "bf16"
    elif case == "f32_r40_unfused":
        dims, R, L, compute = [(20, 30, 40)] * 2, 40, (10, 0, 0), "f32"
    else:
        dims, R, L, compute = [(24, 40, 33), (24, 17, 50), (24, 29, 8)], 12, (6, 0, 0), "f32"
    dt = np.float64 if compute == "f64" else np.float32
    P = synth.coupled_problem(dims, R, L, 10.0, 931, dtype=dt)
    U0, lam0 = synth.uniform_init(P.dims, R, L, 932)
    kw = {} if cb is None else {"coupled_blocks": cb}
    a = model(P, U0, lam0, compute=compute, **kw)
    b = model(P, U0, lam0, compute=compute, **kw)
    if compute == "bf16":
        a.set_option("p1_dma", 1)
        b.set_option("p1_dma", 1)
    a.set_option("fuse", 0)
    b.set_option("fuse", 1)
    assert a.get_option("fuse") == 0
    assert b.get_option("fuse") == 1
    for it in range(3):
        sa, sb = a.step(3), b.step(3)
        say(f"   after {3 * (it + 1)}: F {sa['F']:.12e} / {sb['F']:.12e}")
        assert sa == sb
        for x, y in zip(factors(a), factors(b)):
            np.testing.assert_array_equal(x, y)
        for s in range(len(dims)):
            np.testing.assert_array_equal(a.lam(s), b.lam(s))
    # profiled fused sweeps repeat the fused launches and leave the iterate alone
    b.profile(True)
    sb = b.step(2)
    b.profile(False)
    sa = a.step(2)
    assert sa == sb
    with pytest.raises(ConcpdError):
        b.set_option("fuse", 2)


def test_fused_launches_match_oracle():
    say("[fuse] against the oracle")
    L = (5, 0, 0)
    P = synth.coupled_problem([(40, 70, 100)] * 3, 20, L, 10.0, 941)
    U0, lam0 = synth.uniform_init(P.dims, 20, L, 942)
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=L), iters=4)
    m = model(P, U0, lam0)
    m.set_option("fuse", 1)
    s = m.step(4)
    e = max(rel(m.factor(n, b), ref.U[n][b]) for n in range(3) for b in range(3))
    emax = max(np.max(np.abs(m.factor(n, b) - ref.U[n][b])) / np.max(np.abs(ref.U[n][b])) for n in range(3) for b in range(3))
    say(f"   F={s['F']:.10e} oracle={ref.F:.10e} factor err={e:.2e} elementwise={emax:.2e}")
    assert abs(s["F"] - ref.F) / ref.F <= 1e-5 and e <= 1e-5 and emax <= 1e-4
