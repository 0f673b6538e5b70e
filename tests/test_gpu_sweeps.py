"""The synthetic experiment's sweeps (Section IV-A, Experiment 1d: noise level,
Experiment 1e: tensor size) as parity tests, at reduced block counts and
sizes: every point runs CoNCPD-APG to the paper's stopping rule
(|RelErr_k - RelErr_{k-1}| < 1e-8 or 1000 iterations) on the GPU and in the
FP64 oracle from the same start, and the final global fits must agree within
1e-3 (the metric's gate).  The lraCoNCPD-APG point compresses each block by the
paper's CPD-ALS (1e-4, 200 iterations) on both sides from the same ALS start,
then runs the same rule against the compressed blocks; its global fit against
the original tensors is compared the same way.

Setting of the sweeps: U[0,1] factors, R = 10, coupling L = [5, 5, 0]
(the first five columns of modes 1 and 2 shared), energy SNR (reading of the
noise formula); the paper's 20 blocks of 100^3 are cut to 6 blocks here so
that the oracle runs each point to convergence in seconds.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import apg, cpals
from oracle.apg import DenseData, Options, TuckerData

pytestmark = pytest.mark.gpu

R, L = 10, (5, 5, 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def model(P, U0, lam0, **kw):
    import torch
    from paper_2302_05119_amd import CoupledCP
    dev = torch.device("cuda:0")
    tens = [torch.from_numpy(np.ascontiguousarray(X)).to(dev) for X in P.tensors]
    return CoupledCP(tens, R, L, compute="f32", init_U=U0, init_lambda=lam0, tol=1e-8, max_it=1000, **kw)


def point(snr, I, seed, lra=False):
    P = synth.coupled_problem([(I, I, I)] * 6, R, L, float(snr), seed, dtype=np.float32)
    U0, lam0 = synth.uniform_init(P.dims, R, L, seed + 1)
    U32 = [[u.astype(np.float32).astype(np.float64) for u in per] for per in U0]
    if not lra:
        ref = apg.run(DenseData(P.tensors), U32, lam0, Options(L=L, tol=1e-8, max_it=1000))
        m = model(P, U0, lam0)
        st = m.fit()
        return P, st, m.global_fit(), apg.fit(P.tensors, ref.lam, ref.U), ref.k
    # CPD-ALS starts drawn by the harness, passed to both sides
    rng = np.random.default_rng(seed + 2)
    init = [[rng.uniform(0.0, 1.0, (I, R)) for _ in range(P.S)] for _ in range(3)]
    facs, its, _ = cpals.compress_all_cp([X.astype(np.float64) for X in P.tensors],
                                         [[init[n][s] for n in range(3)] for s in range(P.S)], 1e-4, 200)
    cores, bases = zip(*[cpals.kruskal_as_tucker(U) for U in facs])
    ref = apg.run(TuckerData(list(cores), list(bases)), U32, lam0, Options(L=L, tol=1e-8, max_it=1000))
    m = model(P, U0, lam0, tucker_ranks=(R, R, R))
    out = m.lra_compress_cp(init=init, eps=1e-4, max_it=200)
    # the ALS stop at eps = 1e-4 compares FP32 RelErr changes with FP64 ones:
    # a block may stop one iteration apart; the gate is the final fit
    assert all(abs(a - b) <= 1 for a, b in zip(out["als_iters"], its)), (out["als_iters"], its)
    st = m.fit()
    return P, st, m.global_fit(), apg.fit(P.tensors, ref.lam, ref.U), ref.k


@pytest.mark.parametrize("snr", [0, 6, 12, 20])
def test_snr_sweep_point_matches_oracle(snr):
    # Experiment 1d at I = 30: the fit rises with the SNR
    P, st, gf, rf, k_ref = point(snr, 30, 4100 + snr)
    say(f"[sweep snr {snr} dB] k gpu={st['k']} oracle={k_ref}; fit gpu={gf:.8f} oracle={rf:.8f}")
    assert 1 <= st["k"] <= 1000 and st["converged"] == int(st["k"] < 1000)
    assert abs(gf - rf) <= 1e-3


@pytest.mark.parametrize("I", [10, 30, 50])
def test_size_sweep_point_matches_oracle(I):
    # Experiment 1e at 20 dB: I = 10 n
    P, st, gf, rf, k_ref = point(20, I, 4200 + I)
    say(f"[sweep size I={I}] k gpu={st['k']} oracle={k_ref}; fit gpu={gf:.8f} oracle={rf:.8f}")
    assert 1 <= st["k"] <= 1000 and st["converged"] == int(st["k"] < 1000)
    assert abs(gf - rf) <= 1e-3


@pytest.mark.parametrize("snr,I", [(6, 30), (20, 40)])
def test_lra_sweep_point_matches_oracle(snr, I):
    P, st, gf, rf, k_ref = point(snr, I, 4300 + snr + I, lra=True)
    say(f"[sweep lra snr {snr} dB I={I}] k gpu={st['k']} oracle={k_ref}; global fit gpu={gf:.8f} oracle={rf:.8f}")
    assert 1 <= st["k"] <= 1000 and st["converged"] == int(st["k"] < 1000)
    assert abs(gf - rf) <= 1e-3


def test_sweep_trend_fit_rises_with_snr():
    # the sweep's shape, not only its points: fits increase with the SNR and
    # sit near the noise floor 1 - rho / sqrt(1 + rho^2), rho = 10^(-SNR/20)
    fits = []
    for snr in (0, 10, 20):
        P, st, gf, rf, _ = point(snr, 20, 4400 + snr)
        rho = 10.0 ** (-snr / 20.0)
        floor = 1.0 - rho / np.sqrt(1.0 + rho * rho)
        say(f"[sweep trend {snr} dB] fit {gf:.6f}, noise floor {floor:.6f}")
        fits.append(gf)
        assert abs(gf - rf) <= 1e-3
        assert gf >= floor - 0.02
    assert fits[0] < fits[1] < fits[2]
