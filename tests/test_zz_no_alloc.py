"""concpd_init_static: the context whose workspace is the library's static
device array (no allocation by the library or the caller) gives the same
iterates as concpd_init with a caller-allocated workspace, on two contexts in
a row on one device, the second on a smaller problem; its rejections."""
import numpy as np
import pytest

import synth
from paper_2302_05119_amd import CoupledCP
from paper_2302_05119_amd._lib import STATIC_WORKSPACE_BYTES, ConcpdError

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _problem(dims, R, L, seed):
    P = synth.coupled_problem(dims, R, L, 10.0, seed, dtype=np.float32)
    U0, lam0 = synth.uniform_init(P.dims, R, L, seed + 1)
    return P, U0, lam0


def _state(m, S):
    U = [[m.factor(n, s) for s in range(S)] for n in range(3)]
    lam = [m.lam(s) for s in range(S)]
    return U, lam


def _run_pair(dims, R, L, seed, iters):
    print(f"static workspace: dims={dims} R={R} L={L} seed={seed} iters={iters}", flush=True)
    P, U0, lam0 = _problem(dims, R, L, seed)
    dev = torch.device("cuda:0")
    tens = [torch.from_numpy(X).to(dev) for X in P.tensors]
    ref = CoupledCP(tens, R, L, compute="f32", init_U=U0, init_lambda=lam0)
    st_ref = ref.step(iters)
    Uref, lref = _state(ref, len(dims))
    ref.close()
    m = CoupledCP(tens, R, L, compute="f32", init_U=U0, init_lambda=lam0, static_workspace=True)
    assert m.workspace is None
    st = m.step(iters)
    U, lam = _state(m, len(dims))
    assert st["k"] == st_ref["k"] == iters
    assert st["restarts"] == st_ref["restarts"]
    # the same kernels on the same inputs in the same order: bit-identical
    # (the FP32 bar of 1e-5 relative would be the fallback claim)
    assert st["F"] == st_ref["F"]
    for s in range(len(dims)):
        assert np.array_equal(lam[s], lref[s])
        for n in range(3):
            assert np.array_equal(U[n][s], Uref[n][s]), (n, s)
    return m


def test_static_workspace_matches_allocated_two_calls():
    m1 = _run_pair([(40, 50, 60), (40, 33, 70), (40, 64, 17)], 8, (3, 0, 0), 301, 6)
    m1.close()
    # a second context on the same device after the first is gone, smaller:
    # the array keeps the first one's contents, which must not leak in
    m2 = _run_pair([(20, 30, 25), (20, 11, 9)], 5, (2, 0, 0), 302, 5)
    m2.close()


def test_static_workspace_rejections():
    dev = torch.device("cuda:0")
    P, U0, lam0 = _problem([(16, 12, 10), (16, 9, 14)], 4, (1, 0, 0), 303)
    tens = [torch.from_numpy(X).to(dev) for X in P.tensors]
    m = CoupledCP(tens, 4, (1, 0, 0), init_U=U0, init_lambda=lam0, static_workspace=True)
    # one context per device at a time
    with pytest.raises(ConcpdError, match="ESTATE"):
        CoupledCP(tens, 4, (1, 0, 0), init_U=U0, init_lambda=lam0, static_workspace=True)
    m.step(2)
    m.close()
    # freed: a new one may take it
    m = CoupledCP(tens, 4, (1, 0, 0), init_U=U0, init_lambda=lam0, static_workspace=True)
    m.close()
    # a configuration whose workspace exceeds the array is refused before any device work
    # (512 x 512 x 8 at R = 40: the mode-3 product alone is 40 MiB)
    big = [torch.ones((512, 512, 8), dtype=torch.float32, device=dev) for _ in range(2)]
    with pytest.raises(ConcpdError, match="EINVAL.*static workspace"):
        CoupledCP(big, 40, (8, 0, 0), static_workspace=True)
    # the same configuration with an allocated workspace is fine
    CoupledCP(big, 40, (8, 0, 0)).close()
    assert STATIC_WORKSPACE_BYTES == 32 << 20
