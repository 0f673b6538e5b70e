"""Seeded synthetic inputs for coupled nonnegative CP decomposition.

This module only draws random numbers and assembles test problems from the
generative model of Section II-C (eq. tensormodel: a sum of R rank-1 terms per
block, the first L_n columns of every mode-n factor shared by all blocks).  It
holds none of the fitting method's arithmetic, so the CPU oracle and the HIP
path can both be fed from it without sharing code.

Every array is produced with NumPy's PCG64 generator from an explicit seed, in
float64, then (unless the workload is float64) rounded to float32.  Both sides
of a parity test consume the rounded values.

Noise follows the energy reading of the paper's SNR formula (Section IV,
"Experiment settings"): ``M + 10**(-snr/20) * ||M||_F * N / ||N||_F`` with N
standard normal.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _shared_columns(rng, S, I, R, L, draw):
    """One I x R factor per block; the first L columns are one common draw."""
    common = draw(rng, I, L)
    out = []
    for _ in range(S):
        own = draw(rng, I, R - L)
        out.append(np.concatenate([common, own], axis=1))
    return out


def _uniform(rng, rows, cols):
    return rng.random((rows, cols))


def cp_tensor(factors: Sequence[np.ndarray], lam=None) -> np.ndarray:
    """Dense N-way tensor sum_r lam_r u1_r o u2_r o ... o uN_r (C-contiguous, float64)."""
    R = factors[0].shape[1]
    w = np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)
    if len(factors) == 3:
        A, B, C = factors
        return np.einsum("ir,jr,kr,r->ijk", A, B, C, w, optimize=True)
    idx = "ijklmn"[:len(factors)]
    spec = ",".join(c + "r" for c in idx) + ",r->" + idx
    return np.einsum(spec, *factors, w, optimize=True)


def add_noise(rng, X: np.ndarray, snr_db: float | None) -> np.ndarray:
    if snr_db is None:
        return X
    noise = rng.standard_normal(X.shape)
    scale = 10.0 ** (-snr_db / 20.0) * np.linalg.norm(X) / np.linalg.norm(noise)
    return X + scale * noise


@dataclass
class Problem:
    dims: List[Tuple[int, ...]]
    R: int
    L: Tuple[int, ...]
    tensors: List[np.ndarray]          # storage dtype (float32 or float64), C-contiguous
    true_factors: List[List[np.ndarray]]  # [n][s], float64
    snr_db: float | None
    meta: dict = field(default_factory=dict)

    @property
    def S(self):
        return len(self.dims)


def coupled_problem(dims, R, L, snr_db, seed, dtype=np.float32, factor_draw=None, block_ranks=None,
                    block_lam=None, noise="gaussian") -> Problem:
    """Blocks M^(s) = [[U^(1,s), ..., U^(N,s)]] (lambda = 1) plus noise.

    ``dims`` is a list of S (I1, ..., IN) (N = 3..6, the N-way model of
    Section II-C); a mode with L_n > 0 must have the same
    size in every block.  Factors are U[0,1] unless ``factor_draw(rng, n, s_or_None,
    rows, cols)`` is given.  ``block_ranks`` (R^(s) <= R) keeps only the first
    R^(s) components of block s; ``block_lam`` = (lo, hi) draws per-block
    component weights U[lo, hi] (kept in ``meta['lam']``).  ``noise`` is
    "gaussian" (energy SNR of ``snr_db``) or "salt_pepper" (the block scaled to
    [0, 1], then a fraction ``snr_db`` of its entries set to 0 or 1).
    """
    rng = rng_for(seed)
    S = len(dims)
    N = len(dims[0])
    truth = []
    for n in range(N):
        sizes = [d[n] for d in dims]
        if L[n] > 0:
            assert len(set(sizes)) == 1, "coupled mode needs equal sizes"
        if factor_draw is None:
            draw = lambda g, rows, cols: _uniform(g, rows, cols)  # noqa: E731
        else:
            draw = lambda g, rows, cols, _n=n: factor_draw(g, _n, rows, cols)  # noqa: E731
        if len(set(sizes)) == 1:
            truth.append(_shared_columns(rng, S, sizes[0], R, L[n], draw))
        else:
            truth.append([draw(rng, sizes[s], R) for s in range(S)])
    meta = {}
    if block_ranks is not None:
        truth = [[u.copy() for u in per] for per in truth]
        for s, r in enumerate(block_ranks):
            for n in range(N):
                truth[n][s][:, r:] = 0.0
        meta["block_ranks"] = [int(r) for r in block_ranks]
    lams = None
    if block_lam is not None:
        lams = [rng.uniform(block_lam[0], block_lam[1], size=R) for _ in range(S)]
        meta["lam"] = lams
    tensors = []
    for s in range(S):
        X = cp_tensor([truth[n][s] for n in range(N)], None if lams is None else lams[s])
        if noise == "salt_pepper":
            X = salt_pepper(rng, X / np.max(X), snr_db)
        else:
            X = add_noise(rng, X, snr_db)
        tensors.append(np.ascontiguousarray(X.astype(dtype)))
    return Problem(list(map(tuple, dims)), R, tuple(L), tensors, truth, snr_db, meta=meta)


def salt_pepper(rng, X: np.ndarray, frac: float) -> np.ndarray:
    """A fraction ``frac`` of the entries set to 0 or 1 (equally likely)."""
    X = X.copy()
    hit = rng.random(X.shape) < frac
    X[hit] = (rng.random(int(hit.sum())) < 0.5).astype(np.float64)
    return X


def eeg_problem(S, T_range, R, snr_db, seed, channels=64, freqs=60, dtype=np.float32) -> Problem:
    """EEG-shaped blocks channel x frequency x time with uneven T_s.

    Topographies |N(0,1)| and spectra (Gaussian bumps) are shared by every block
    (L = [R, R, 0]); temporal courses are |AR(1)| with phi = 0.9 per block.
    """
    rng = rng_for(seed)
    T = rng.integers(T_range[0], T_range[1] + 1, size=S)
    topo = np.abs(rng.standard_normal((channels, R)))
    f = np.arange(freqs, dtype=np.float64)[:, None]
    c = rng.uniform(0, freqs - 1, size=R)[None, :]
    sig = rng.uniform(2.0, 8.0, size=R)[None, :]
    spec = np.exp(-((f - c) ** 2) / (2 * sig ** 2))
    phi = 0.9
    temporal = []
    for s in range(S):
        e = rng.standard_normal((int(T[s]), R))
        x = np.empty_like(e)
        x[0] = e[0] / np.sqrt(1 - phi * phi)
        for t in range(1, int(T[s])):
            x[t] = phi * x[t - 1] + e[t]
        temporal.append(np.abs(x))
    truth = [[topo] * S, [spec] * S, temporal]
    tensors = []
    for s in range(S):
        X = cp_tensor([topo, spec, temporal[s]])
        X = add_noise(rng, X, snr_db)
        tensors.append(np.ascontiguousarray(X.astype(dtype)))
    dims = [(channels, freqs, int(T[s])) for s in range(S)]
    return Problem(dims, R, (R, R, 0), tensors, truth, snr_db, meta={"T": T.tolist()})


def uniform_init(dims, R, L, seed):
    """Seeded U[0,1] initial factors [n][s] (shared columns drawn once) and
    lambda^(s) ~ U[0,1]^R, all float64 (the paper initialises with MATLAB rand)."""
    rng = rng_for(seed)
    S = len(dims)
    U = []
    for n in range(len(dims[0])):
        sizes = [d[n] for d in dims]
        if len(set(sizes)) == 1:
            U.append(_shared_columns(rng, S, sizes[0], R, L[n], _uniform))
        else:
            U.append([_uniform(rng, sizes[s], R) for s in range(S)])
    lam = [rng.random(R) for _ in range(S)]
    return U, lam


def downsample(problem: Problem, step: int) -> Problem:
    """Slice-downsampled copy M[::step, ::step, ::step] (keeps the CP + noise form)."""
    tensors = [np.ascontiguousarray(X[::step, ::step, ::step]) for X in problem.tensors]
    dims = [t.shape for t in tensors]
    truth = [[U[::step] for U in per_mode] for per_mode in problem.true_factors]
    return Problem(dims, problem.R, problem.L, tensors, truth, problem.snr_db,
                   meta=dict(problem.meta, downsample=step))


# ---------------------------------------------------------------------------
# Workloads.  Sizes follow the experiments of Section IV (synthetic 100^3,
# EEG-shaped channel x frequency x time) scaled to one GPU.
# ---------------------------------------------------------------------------
WORKLOADS = {
    "c1_fp64_2x30cube_r5": dict(dims=[(30, 30, 30)] * 2, R=5, L=(5, 0, 0), snr=20.0,
                                iters=50, dtype="f64", seed=1001),
    "c2_fp32_10x100cube_r20": dict(dims=[(100, 100, 100)] * 10, R=20, L=(5, 0, 0), snr=10.0,
                                   iters=200, dtype="f32", seed=1002),
    "c3_lra_10x256cube_r20": dict(dims=[(256, 256, 256)] * 10, R=20, L=(8, 0, 0), snr=20.0,
                                  iters=300, dtype="f32", seed=1003, tucker=(30, 30, 30)),
    "c4_eeg_bf16_16blocks_r30": dict(S=16, T_range=(200, 2000), R=30, L=(30, 30, 0), snr=5.0,
                                     iters=200, dtype="bf16", seed=1004),
    "c5_lra_4x512cube_r40": dict(dims=[(512, 512, 512)] * 4, R=40, L=(40, 0, 0), snr=15.0,
                                 iters=500, dtype="f32", seed=1005, tucker=(40, 40, 40)),
    # face-image-shaped (Section IV, Experiment 2): 31 subjects of 32 x 32 pixels x
    # 64 illuminations, per-subject ranks 22..26, 15 components coupled in the two
    # pixel modes, salt-and-pepper noise on the [0, 1]-scaled blocks
    "face_31x32x32x64_r22to26": dict(dims=[(32, 32, 64)] * 31, R=26, L=(15, 15, 0), snr=0.1,
                                     noise="salt_pepper", rank_range=(22, 26), iters=200, dtype="f32", seed=1006),
    # ERP-shaped (Section IV, Experiment 3): 42 subjects of 9 channels x 71
    # frequency bins x 60 time points, R = 36 coupled in every mode; the blocks
    # differ only through their core weights (drawn U[0.5, 1.5] per component)
    "erp_42x9x71x60_r36_full": dict(dims=[(9, 71, 60)] * 42, R=36, L=(36, 36, 36), snr=10.0,
                                    block_lam=(0.5, 1.5), iters=200, dtype="f32", seed=1007),
    # the N-way model (Section II-C) at N = 4 with the byte count of the
    # 10 x 100^3 case: 10 blocks of 32^4, R = 20, five shared mode-1 columns
    "n4_fp32_10x32x4_r20": dict(dims=[(32, 32, 32, 32)] * 10, R=20, L=(5, 0, 0, 0), snr=10.0,
                                iters=200, dtype="f32", seed=1008),
}


def make_workload(name: str, dtype=None) -> Problem:
    w = WORKLOADS[name]
    if name.startswith("c4"):
        return eeg_problem(w["S"], w["T_range"], w["R"], w["snr"], w["seed"],
                           dtype=dtype or np.float32)
    store = dtype or (np.float64 if w["dtype"] == "f64" else np.float32)
    ranks = None
    if "rank_range" in w:
        lo, hi = w["rank_range"]
        ranks = rng_for(w["seed"] + 500).integers(lo, hi + 1, size=len(w["dims"])).tolist()
    return coupled_problem(w["dims"], w["R"], w["L"], w["snr"], w["seed"], dtype=store, block_ranks=ranks,
                           block_lam=w.get("block_lam"), noise=w.get("noise", "gaussian"))


def workload_init(name: str, problem: Problem):
    """U[0,1] start [n][s] and lambda [s]; with per-block ranks, block s keeps
    its first R^(s) columns."""
    w = WORKLOADS[name]
    U, lam = uniform_init(problem.dims, problem.R, problem.L, w["seed"] + 1000)
    ranks = problem.meta.get("block_ranks")
    if ranks is not None:
        U = [[u[:, :ranks[s]].copy() for s, u in enumerate(per)] for per in U]
        lam = [l[:ranks[s]].copy() for s, l in enumerate(lam)]
    return U, lam
