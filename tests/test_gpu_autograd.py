"""The autograd form: concpd_loss_grad and the torch.autograd.Function.

The loss and every gradient are compared with the FP64 oracle's
loss_and_grads at points that are not APG iterates (FP64 path <= 1e-10,
FP32 path <= 1e-5 normwise relative), against central finite differences of
the library's own FP64 loss, and through torch.autograd with tied shared
columns (autograd's sum over blocks must equal the oracle's coupled gradient).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import apg
from oracle.apg import DenseData

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / n if n > 0 else np.linalg.norm(a - b)


def setup(compute, L=(2, 0, 1), R=5, seed=701):
    import torch
    from paper_2302_05119_amd import CoupledCP
    dtype = np.float64 if compute == "f64" else np.float32
    P = synth.coupled_problem([(20, 30, 25), (20, 18, 25), (20, 11, 25)], R, L, 10.0, seed, dtype=dtype)
    dev = torch.device("cuda:0")
    tens = [torch.from_numpy(np.ascontiguousarray(X)).to(dev) for X in P.tensors]
    m = CoupledCP(tens, R, L, compute=compute, seed=3)
    # a point that is not an iterate: fresh U[0,1] factors (shared columns
    # drawn once) and lambda in [0.5, 1.5]
    U, lam = synth.uniform_init(P.dims, R, L, seed + 1)
    lam = [l + 0.5 for l in lam]
    if compute != "f64":
        U = [[u.astype(np.float32).astype(np.float64) for u in per] for per in U]
    return P, m, U, lam, dev


def to_dev(U, lam, compute, dev, requires_grad=False):
    import torch
    ft = torch.float64 if compute == "f64" else torch.float32
    Ut = [[torch.tensor(u, dtype=ft, device=dev, requires_grad=requires_grad) for u in per] for per in U]
    lt = [torch.tensor(l, dtype=torch.float64, device=dev, requires_grad=requires_grad) for l in lam]
    return Ut, lt


@pytest.mark.parametrize("compute,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_loss_and_gradients_match_oracle(compute, tol):
    say(f"[loss_grad] compute={compute}")
    P, m, U, lam, dev = setup(compute)
    F_ref, gl_ref, gU_ref, gC_ref = apg.loss_and_grads(DenseData(P.tensors), lam, U, P.L)
    Ut, lt = to_dev(U, lam, compute, dev)
    for coupled in (False, True):
        F, gU, gl = m.loss_grad(Ut, lt, coupled=coupled)
        say(f"   coupled={coupled} F gpu={F:.15e} oracle={F_ref:.15e}")
        assert abs(F - F_ref) / F_ref <= tol
        for s in range(P.S):
            assert rel(gl[s].cpu().numpy(), gl_ref[s]) <= tol
            for n in range(3):
                g = gU[n][s].cpu().numpy()
                Ln = P.L[n]
                e = rel(g[:, Ln:], gU_ref[n][s][:, Ln:]) if Ln < P.R else 0.0
                assert e <= tol, (coupled, n, s, e)
                if Ln > 0:
                    want = gC_ref[n] if coupled else gU_ref[n][s][:, :Ln]
                    assert rel(g[:, :Ln], want) <= tol, (coupled, n, s)


def test_gradient_matches_finite_differences():
    import torch
    say("[loss_grad] finite differences (FP64)")
    P, m, U, lam, dev = setup("f64", seed=711)
    Ut, lt = to_dev(U, lam, "f64", dev)
    F0, gU, gl = m.loss_grad(Ut, lt)
    rng = np.random.default_rng(5)
    for trial in range(3):
        dU = [[torch.tensor(rng.standard_normal(u.shape), device=dev) for u in per] for per in Ut]
        dl = [torch.tensor(rng.standard_normal(l.shape), device=dev) for l in lt]
        h = 1e-5
        Fp, _, _ = m.loss_grad([[u + h * d for u, d in zip(pu, pd)] for pu, pd in zip(Ut, dU)],
                               [l + h * d for l, d in zip(lt, dl)])
        Fm, _, _ = m.loss_grad([[u - h * d for u, d in zip(pu, pd)] for pu, pd in zip(Ut, dU)],
                               [l - h * d for l, d in zip(lt, dl)])
        fd = (Fp - Fm) / (2 * h)
        an = sum(float((g * d).sum()) for pg, pd in zip(gU, dU) for g, d in zip(pg, pd))
        an += sum(float((g * d).sum()) for g, d in zip(gl, dl))
        say(f"   trial {trial}: fd={fd:.12e} analytic={an:.12e}")
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1.0)


def test_autograd_function_with_tied_shared_columns():
    import torch
    from paper_2302_05119_amd import coupled_cp_loss
    say("[autograd] tied shared columns")
    P, m, U, lam, dev = setup("f64", seed=721)
    F_ref, gl_ref, gU_ref, gC_ref = apg.loss_and_grads(DenseData(P.tensors), lam, U, P.L)
    shared = [torch.tensor(U[n][0][:, :P.L[n]], device=dev, requires_grad=True) if P.L[n] > 0 else None for n in range(3)]
    indiv = [[torch.tensor(U[n][s][:, P.L[n]:], device=dev, requires_grad=True) for s in range(P.S)] for n in range(3)]
    Ut = [[torch.cat([shared[n], indiv[n][s]], dim=1) if P.L[n] > 0 else indiv[n][s] for s in range(P.S)]
          for n in range(3)]
    lt = [torch.tensor(l, device=dev, requires_grad=True) for l in lam]
    loss = coupled_cp_loss(m, Ut, lt)
    (2.0 * loss).backward()
    say(f"   loss={loss.item():.12e} oracle={F_ref:.12e}")
    assert abs(loss.item() - F_ref) / F_ref <= 1e-10
    for n in range(3):
        if P.L[n] > 0:
            assert rel(shared[n].grad.cpu().numpy(), 2.0 * gC_ref[n]) <= 1e-10
        for s in range(P.S):
            assert rel(indiv[n][s].grad.cpu().numpy(), 2.0 * gU_ref[n][s][:, P.L[n]:]) <= 1e-10
    for s in range(P.S):
        assert rel(lt[s].grad.cpu().numpy(), 2.0 * gl_ref[s]) <= 1e-10


def test_autograd_gradcheck_small():
    import torch
    from paper_2302_05119_amd import CoupledCP, CoupledCPLoss
    say("[autograd] gradcheck")
    P = synth.coupled_problem([(4, 5, 3), (4, 3, 3)], 2, (1, 0, 0), 10.0, 731, dtype=np.float64)
    dev = torch.device("cuda:0")
    m = CoupledCP([torch.from_numpy(X).to(dev) for X in P.tensors], 2, (1, 0, 0), compute="f64", seed=1)
    U, lam = synth.uniform_init(P.dims, 2, (1, 0, 0), 732)
    params = [torch.tensor(U[n][s], device=dev, requires_grad=True) for n in range(3) for s in range(2)]
    params += [torch.tensor(l + 0.5, device=dev, requires_grad=True) for l in lam]
    assert torch.autograd.gradcheck(lambda *p: CoupledCPLoss.apply(m, *p), params, eps=1e-6, atol=1e-6, rtol=1e-5)


def test_loss_grad_leaves_the_iterate_alone():
    import torch
    from paper_2302_05119_amd import CoupledCP
    say("[loss_grad] iterate untouched")
    P, m, U, lam, dev = setup("f32", seed=741)
    tens = [torch.from_numpy(np.ascontiguousarray(X)).to(dev) for X in P.tensors]
    m2 = CoupledCP(tens, P.R, P.L, compute="f32", seed=3)
    m.step(3)
    m2.step(3)
    Ut, lt = to_dev(U, lam, "f32", dev)
    m.loss_grad(Ut, lt)
    s1, s2 = m.step(2), m2.step(2)
    assert s1["k"] == s2["k"] == 5 and s1["F"] == s2["F"]
    for n in range(3):
        for s in range(P.S):
            np.testing.assert_array_equal(m.factor(n, s), m2.factor(n, s))


@pytest.mark.parametrize("compute,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_loss_and_gradients_with_coupling_groups(compute, tol):
    # flexible coupling (Section III-C): mode 1 shared by blocks 0 and 2 only,
    # mode 3 by blocks 1 and 2; the shared gradient is the group's sum
    import torch
    from paper_2302_05119_amd import CoupledCP
    say(f"[loss_grad] coupling groups compute={compute}")
    dtype = np.float64 if compute == "f64" else np.float32
    L, R, groups = (2, 0, 1), 4, ((0, 2), None, (1, 2))
    P = synth.coupled_problem([(9, 10, 11), (7, 12, 11), (9, 8, 11)], R, (0, 0, 0), 10.0, 741, dtype=dtype)
    dev = torch.device("cuda:0")
    m = CoupledCP([torch.from_numpy(X).to(dev) for X in P.tensors], R, L, compute=compute, seed=3,
                  coupled_blocks=groups)
    rng = np.random.default_rng(742)
    U = [[rng.random((d[n], R)) for d in P.dims] for n in range(3)]
    for n, grp in ((0, groups[0]), (2, groups[2])):
        for b in grp[1:]:
            U[n][b][:, :L[n]] = U[n][grp[0]][:, :L[n]]
    if compute != "f64":
        U = [[u.astype(np.float32).astype(np.float64) for u in per] for per in U]
    lam = [rng.random(R) + 0.5 for _ in range(P.S)]
    F_ref, gl_ref, gU_ref, gC_ref = apg.loss_and_grads(DenseData(P.tensors), lam, U, L, coupled_blocks=groups)
    Ut, lt = to_dev(U, lam, compute, dev)
    F, gU, gl = m.loss_grad(Ut, lt, coupled=True)
    say(f"   F gpu={F:.15e} oracle={F_ref:.15e}")
    assert abs(F - F_ref) / F_ref <= tol
    for s in range(P.S):
        assert rel(gl[s].cpu().numpy(), gl_ref[s]) <= tol
        for n in range(3):
            g = gU[n][s].cpu().numpy()
            member = L[n] > 0 and s in (groups[n] or range(P.S))
            Ls = L[n] if member else 0
            assert rel(g[:, Ls:], gU_ref[n][s][:, Ls:]) <= tol, (n, s)
            if member:
                assert rel(g[:, :Ls], gC_ref[n]) <= tol, (n, s)


def bf16_round(X):
    """FP32 values rounded to the nearest BF16 (ties to even), as FP64."""
    b = np.ascontiguousarray(X, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def test_loss_grad_bf16_full_eeg_workload():
    # the autograd form at its own configuration: 16 EEG-shaped blocks
    # (64 x 60 x T_s, T_s ~ U{200..2000}), R = 30, channel and frequency
    # factors fully coupled, BF16 tensor operands.  Against the FP64 oracle on
    # the FP32 tensors: 2e-2 normwise and elementwise-max (the per-step BF16
    # bound); against the oracle on the BF16-rounded tensors: 1e-5 (what is
    # left is FP32 accumulation).
    import torch
    from paper_2302_05119_amd import CoupledCP
    say("[loss_grad] BF16, full 16-block EEG-shaped workload")
    P = synth.make_workload("c4_eeg_bf16_16blocks_r30")
    dev = torch.device("cuda:0")
    tens = [torch.from_numpy(np.ascontiguousarray(X)).to(dev) for X in P.tensors]
    m = CoupledCP(tens, P.R, P.L, compute="bf16", seed=5)
    U, lam = synth.uniform_init(P.dims, P.R, P.L, 1741)
    lam = [l + 0.5 for l in lam]
    U = [[u.astype(np.float32).astype(np.float64) for u in per] for per in U]
    Ut, lt = to_dev(U, lam, "bf16", dev)
    ref32 = apg.loss_and_grads(DenseData(P.tensors), lam, U, P.L)
    ref16 = apg.loss_and_grads(DenseData([bf16_round(X) for X in P.tensors]), lam, U, P.L)
    for coupled in (False, True):
        F, gU, gl = m.loss_grad(Ut, lt, coupled=coupled)
        for name, (F_ref, gl_ref, gU_ref, gC_ref), tol in (("fp32 data", ref32, 2e-2), ("bf16 data", ref16, 1e-5)):
            eF = abs(F - F_ref) / F_ref
            worst = (eF, 0.0)
            for s in range(P.S):
                worst = max(worst, (rel(gl[s].cpu().numpy(), gl_ref[s]), maxrel(gl[s].cpu().numpy(), gl_ref[s])))
                for n in range(3):
                    g = gU[n][s].cpu().numpy().astype(np.float64)
                    want = gU_ref[n][s].copy()
                    if coupled and P.L[n] > 0:
                        want[:, :P.L[n]] = gC_ref[n]
                    worst = max(worst, (rel(g, want), maxrel(g, want)))
            say(f"   coupled={coupled} vs oracle on {name}: F rel {eF:.2e}, worst gradient normwise/elementwise "
                f"{worst[0]:.2e} / {worst[1]:.2e}")
            assert eF <= tol and worst[0] <= tol and worst[1] <= (tol if tol >= 1e-3 else 1e-3)


def test_loss_grad_bf16_finite_differences():
    # central differences of the library's own BF16 loss along random
    # directions, against its gradient (EEG-shaped small case)
    import torch
    from paper_2302_05119_amd import CoupledCP
    say("[loss_grad] BF16 finite differences")
    P = synth.eeg_problem(4, (20, 60), 6, 5.0, 1751, channels=16, freqs=12)
    dev = torch.device("cuda:0")
    tens = [torch.from_numpy(np.ascontiguousarray(X)).to(dev) for X in P.tensors]
    m = CoupledCP(tens, P.R, P.L, compute="bf16", seed=5)
    U, lam = synth.uniform_init(P.dims, P.R, P.L, 1752)
    lam = [l + 0.5 for l in lam]
    Ut, lt = to_dev(U, lam, "bf16", dev)
    F0, gU, gl = m.loss_grad(Ut, lt)
    rng = np.random.default_rng(9)
    h = 1e-2
    for trial in range(3):
        dU = [[torch.tensor(rng.standard_normal(u.shape), dtype=torch.float32, device=dev) for u in per] for per in Ut]
        dl = [torch.tensor(rng.standard_normal(l.shape), device=dev) for l in lt]
        Up = [[u + h * d for u, d in zip(pu, pd)] for pu, pd in zip(Ut, dU)]
        Um = [[u - h * d for u, d in zip(pu, pd)] for pu, pd in zip(Ut, dU)]
        Fp, _, _ = m.loss_grad(Up, [l + h * d for l, d in zip(lt, dl)])
        Fm, _, _ = m.loss_grad(Um, [l - h * d for l, d in zip(lt, dl)])
        fd = (Fp - Fm) / 2
        # the FP32 steps actually taken (u + h d rounds), so only the loss's own
        # accuracy and the O(h^2) term remain
        an = sum(float(((up - um).double() * g.double()).sum()) / 2 for pg, pu_, pm_ in zip(gU, Up, Um)
                 for g, up, um in zip(pg, pu_, pm_))
        an += sum(float((g * d).sum()) * h for g, d in zip(gl, dl))
        say(f"   trial {trial}: fd={fd:.10e} analytic={an:.10e}")
        assert abs(fd - an) <= 2e-3 * abs(an)
