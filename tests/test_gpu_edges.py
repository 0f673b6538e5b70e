"""Edge cases of the configuration space through the C ABI, each one
teacher-forced iteration against the FP64 oracle (1e-5 FP32, 1e-10 FP64):
the largest rank (R = 64: sixteen 4-column MFMA tiles, the Lanczos class of
the spectral norm; R = 32 on the FP64 path, its largest), the largest block
count (S = 64), single-element modes
(I_n = 1, and a 1 x 1 x 1 block), rank one with every mode fully shared, and
one block."""
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
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / n if n > 0 else np.linalg.norm(a - b)


CASES = [
    # name, dims, R, L, compute
    ("rank64", [(20, 70, 33), (20, 45, 40)], 64, (10, 0, 0), "f32"),
    ("rank32_f64", [(9, 17, 21)], 32, (0, 0, 0), "f64"),
    ("blocks64", [(5, 6, 7)] * 64, 3, (2, 0, 1), "f32"),
    ("unit_modes", [(1, 5, 7), (6, 1, 9), (4, 8, 1), (1, 1, 1)], 2, (0, 0, 0), "f32"),
    ("unit_modes_f64", [(1, 5, 7), (6, 1, 9), (4, 8, 1), (1, 1, 1)], 2, (0, 0, 0), "f64"),
    ("rank1_full", [(8, 9, 10)] * 3, 1, (1, 1, 1), "f32"),
    ("one_block", [(33, 70, 130)], 9, (0, 0, 0), "f32"),
]


@pytest.mark.parametrize("name,dims,R,L,compute", CASES, ids=[c[0] for c in CASES])
def test_edge_one_iteration_teacher_forced(dev, name, dims, R, L, compute):
    import torch
    from paper_2302_05119_amd import CoupledCP
    say(f"[edge] {name}: S={len(dims)} dims={dims[:4]} R={R} L={L} compute={compute}")
    dtype = np.float64 if compute == "f64" else np.float32
    tol = 1e-10 if compute == "f64" else 1e-5
    P = synth.coupled_problem(dims, R, L, 10.0, 801 + R, dtype=dtype)
    U0, lam0 = synth.uniform_init(P.dims, R, L, 802 + R)
    data = DenseData(P.tensors)
    opt = Options(L=L)
    st = apg.run(data, U0, lam0, opt, iters=2)
    st = copy.deepcopy(st)
    if compute != "f64":
        st.U = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U]
        st.U_prev = [[u.astype(np.float32).astype(np.float64) for u in per] for per in st.U_prev]
    st.F = apg.objective(data, st.lam, st.U)
    tens = [torch.from_numpy(X).to(dev) for X in P.tensors]
    m = CoupledCP(tens, R, L, compute=compute, init_U=st.U, init_lambda=st.lam)
    Lu_prev = [[st.Lu_prev[n][s] for n in range(3)] for s in range(P.S)]
    m.set_state(st.U, st.lam, st.U_prev, st.lam_prev, st.Ld_prev, Lu_prev, st.LC_prev, t=st.t, k=st.k)
    new = apg.iterate(data, st, opt)
    s1 = m.step(1)
    say(f"   F gpu={s1['F']:.12e} oracle={new.F:.12e} restart gpu={s1['restarted_last']} oracle={new.last_restarted}")
    assert bool(s1["restarted_last"]) == bool(new.last_restarted)
    assert abs(s1["F"] - new.F) / new.F <= tol
    Ld, Lu, LC = m.lipschitz()
    ltol = 1e-6 if compute == "f32" else 1e-11
    np.testing.assert_allclose(Ld, new.Ld_prev, rtol=ltol)
    worst = 0.0
    for s in range(P.S):
        np.testing.assert_allclose(Lu[s], [new.Lu_prev[n][s] for n in range(3)], rtol=ltol)
        worst = max(worst, rel(m.lam(s), new.lam[s]))
        for n in range(3):
            worst = max(worst, rel(m.factor(n, s), new.U[n][s]))
    say(f"   worst relative error {worst:.2e}")
    assert worst <= tol
