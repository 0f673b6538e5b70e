"""The paper's second workload shapes (Section IV, Experiments 2 and 3) as
synthetic stand-ins, through the C ABI against the FP64 oracle, at full size:

* face-image-shaped: 31 blocks of 32 x 32 x 64, per-block ranks 22..26 (the
  library's zero-padded R = 26), 15 components coupled in the two pixel modes,
  salt-and-pepper noise;
* ERP-shaped: 42 blocks of 9 x 71 x 60, R = 36 coupled in all three modes (the
  blocks differ only through their cores), which runs the FP64 matrix-core
  spectral-norm class and the coupled sums over 42 blocks.

Teacher-forced single iterations at 1e-5 (FP32 operands), trajectories by fit
at 1e-4.
"""
import copy
import sys

import numpy as np
import pytest

import synth
from oracle import apg
from oracle.apg import DenseData, Options

pytestmark = pytest.mark.gpu

NAMES = ["face_31x32x32x64_r22to26", "erp_42x9x71x60_r36_full"]


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
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / n if n > 0 else np.linalg.norm(a - b)


def make_model(P, U, lam, dev):
    import torch
    from paper_2302_05119_amd import CoupledCP
    tens = [torch.from_numpy(X).to(dev) for X in P.tensors]
    return CoupledCP(tens, P.R, P.L, compute="f32", init_U=U, init_lambda=lam,
                     block_ranks=P.meta.get("block_ranks"))


@pytest.mark.parametrize("name", NAMES)
def test_workload_one_iteration_teacher_forced(dev, name):
    say(f"[workload] {name} teacher-forced")
    P = synth.make_workload(name)
    U0, lam0 = synth.workload_init(name, P)
    data = DenseData(P.tensors)
    opt = Options(L=P.L)
    st = apg.run(data, U0, lam0, opt, iters=2)
    st = copy.deepcopy(st)
    st.U = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U]
    st.U_prev = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U_prev]
    st.F = apg.objective(data, st.lam, st.U)
    m = make_model(P, st.U, st.lam, dev)
    Lu_prev = [[st.Lu_prev[n][s] for n in range(3)] for s in range(P.S)]
    m.set_state(st.U, st.lam, st.U_prev, st.lam_prev, st.Ld_prev, Lu_prev, st.LC_prev, t=st.t, k=st.k)
    new = apg.iterate(data, st, opt)
    s1 = m.step(1)
    say(f"   F gpu={s1['F']:.10e} oracle={new.F:.10e} restart gpu={s1['restarted_last']} oracle={new.last_restarted}")
    assert bool(s1["restarted_last"]) == bool(new.last_restarted)
    assert abs(s1["F"] - new.F) / new.F <= 1e-5
    Ld, Lu, LC = m.lipschitz()
    np.testing.assert_allclose(Ld, new.Ld_prev, rtol=1e-6)
    np.testing.assert_allclose(LC, new.LC_prev, rtol=1e-6)
    worst = 0.0
    for s in range(P.S):
        worst = max(worst, rel(m.lam(s), new.lam[s]))
        for n in range(3):
            worst = max(worst, rel(m.factor(n, s), new.U[n][s]))
    say(f"   worst relative error {worst:.2e}")
    assert worst <= 1e-5


@pytest.mark.parametrize("name", NAMES)
def test_workload_trajectory_fit(dev, name):
    say(f"[workload] {name} 30 iterations")
    P = synth.make_workload(name)
    U0, lam0 = synth.workload_init(name, P)
    m = make_model(P, U0, lam0, dev)
    ref = apg.run(DenseData(P.tensors), U0, lam0, Options(L=P.L), iters=30)
    s = m.step(30)
    gf = m.global_fit()
    rf = apg.fit(P.tensors, ref.lam, ref.U)
    say(f"   fit gpu={gf:.8f} oracle={rf:.8f} restarts {s['restarts']} vs {ref.restarts}")
    assert abs(gf - rf) <= 1e-4
    if P.L == (P.R, P.R, P.R):
        # fully coupled: every factor identical across blocks; only the cores differ
        for n in range(3):
            for b in range(1, P.S):
                np.testing.assert_array_equal(m.factor(n, b), m.factor(n, 0))
