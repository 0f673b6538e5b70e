"""Plain, slow FP64 CPU oracle for CoNCPD-APG (Algorithm 1) and its
low-rank-approximation variant (Algorithm 2).

TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code with
the HIP path and imports nothing from it.

Everything is written in the paper's own formulation (Section III-A and
Appendix A): explicit mode-n unfoldings, explicit Khatri-Rao products, matrix
products, Hadamard products of Grams, ``numpy.linalg.eigvalsh`` for spectral
norms.  No blocking, fusion or reordering beyond those definitions.

Readings of points the paper leaves open (also listed in the design notes):

* Block order is Gauss-Seidel (Section III-A, the paragraph after
  eq. eqextraPU): D^(1..S), then U^(1,1..S), ..., U^(N,1..S); every update sees
  the latest value of every other block.
* A mode-n update first evaluates all S block gradients at the extrapolated
  point, then applies eq. solUnC to the shared columns and eq. solUnsI to each
  individual part (eq. solUnC needs the sum over s of the shared gradients).
* The shared block U_C^(n) is extrapolated with
  w = min(w_hat, delta_w * sqrt(L_C,prev / L_C)), L_C = sum_s L_u^(n,s), the
  same step length that eq. solUnC uses.
* Restart (Algorithm 1): if F_k >= F_{k-1} the whole sweep is redone from
  x_{k-1} with every extrapolation weight 0 and accepted unconditionally; t_k
  keeps running unless ``reset_t`` is set.
* A block whose Lipschitz constant is exactly 0 is left unchanged.
* max(0, .) propagates NaN (np.maximum).
* No column normalisation of the iterates.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# ---------------------------------------------------------------------------
# Tensor algebra of Section II (Table I notation)
# ---------------------------------------------------------------------------


def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n matricization X_(n): rows indexed by i_n, columns by the other
    indices with the lowest mode varying fastest."""
    return np.reshape(np.moveaxis(X, n, 0), (X.shape[n], -1), order="F")


def fold(Xn: np.ndarray, n: int, shape) -> np.ndarray:
    """Inverse of :func:`unfold`."""
    rest = [shape[m] for m in range(len(shape)) if m != n]
    Y = np.reshape(Xn, [shape[n]] + rest, order="F")
    return np.moveaxis(Y, 0, n)


def vec(X: np.ndarray) -> np.ndarray:
    """vec(X): the first index varies fastest."""
    return np.reshape(X, -1, order="F")


def khatri_rao(mats) -> np.ndarray:
    """Column-wise Kronecker product A ⊙ B ⊙ ... (the rightmost factor's row
    index varies fastest)."""
    out = mats[0]
    for B in mats[1:]:
        out = (out[:, None, :] * B[None, :, :]).reshape(-1, out.shape[1])
    return out


def krp_all(U) -> np.ndarray:
    """U^⊙ = U^(N) ⊙ ... ⊙ U^(1)  (Table I)."""
    return khatri_rao(list(U)[::-1])


def krp_minus(U, n: int) -> np.ndarray:
    """U^{⊙-n} = U^(N) ⊙ ... ⊙ U^(n+1) ⊙ U^(n-1) ⊙ ... ⊙ U^(1)  (Table I)."""
    return khatri_rao([U[m] for m in reversed(range(len(U))) if m != n])


def mode_product(X: np.ndarray, B: np.ndarray, n: int) -> np.ndarray:
    """n-mode product X x_n B:  (X x_n B)_(n) = B X_(n)."""
    shape = list(X.shape)
    shape[n] = B.shape[0]
    return fold(B @ unfold(X, n), n, shape)


def hadamard_of_grams(U, skip: Optional[int] = None) -> np.ndarray:
    """(U^T U)^⊛ or, with ``skip = n``, (U^T U)^{⊛-n}: the Hadamard product of
    the factor Grams (Table timecomplx, operations 1 and 4)."""
    R = U[0].shape[1]
    H = np.ones((R, R))
    for m, Um in enumerate(U):
        if m != skip:
            H = H * (Um.T @ Um)
    return H


def spectral_norm(A: np.ndarray) -> float:
    """||A||_2 of a symmetric PSD matrix: its largest eigenvalue (Appendix A,
    eq. eqLipsLd / eqLipsLu)."""
    if A.size == 0:
        return 0.0
    return float(max(0.0, np.linalg.eigvalsh(A)[-1]))


def mttkrp(X: np.ndarray, U, n: int) -> np.ndarray:
    """M_(n) U^{⊙-n}: the data term of eq. solapgU (operations 6 and 7)."""
    return unfold(X, n) @ krp_minus(U, n)


def core_data_term(X: np.ndarray, U) -> np.ndarray:
    """(U^⊙)^T vec(M): the data term of eq. solapgG (operations 2 and 3)."""
    return krp_all(U).T @ vec(X)


def reconstruct(lam: np.ndarray, U) -> np.ndarray:
    """[[D; U^(1), ..., U^(N)]] with D super-diagonal holding lam
    (eq. tensormodel): mode-1 unfolding U^(1) D (U^{⊙-1})^T, folded back."""
    shape = [Um.shape[0] for Um in U]
    X1 = (U[0] * lam[None, :]) @ krp_minus(U, 0).T
    return fold(X1, 0, shape)


# ---------------------------------------------------------------------------
# Extrapolation weights (Appendix A, "Parameter settings")
# ---------------------------------------------------------------------------


def t_next(t_prev: float) -> float:
    """t_k = (1 + sqrt(1 + 4 t_{k-1}^2)) / 2, t_0 = 1."""
    return 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t_prev * t_prev))


def extrapolation_weight(w_hat: float, L_prev, L_cur: float, delta_w: float) -> float:
    """w = min(w_hat_{k-1}, delta_w sqrt(L_{k-2} / L_{k-1}))  (eq. eqextrawd/eqextrawu).
    No previous constant (first iteration) or L_cur = 0 gives w = 0."""
    if L_prev is None or L_cur <= 0.0:
        return 0.0
    return float(min(w_hat, delta_w * np.sqrt(L_prev / L_cur)))


# ---------------------------------------------------------------------------
# Data terms: the original tensors (Algorithm 1) or a compressed form (Algorithm 2)
# ---------------------------------------------------------------------------


class DenseData:
    """Block tensors M^(s) held explicitly."""

    def __init__(self, tensors):
        self.X = [np.asarray(t, dtype=np.float64) for t in tensors]

    @property
    def S(self):
        return len(self.X)

    def shape(self, s):
        return self.X[s].shape

    def mttkrp(self, s, U, n):
        return mttkrp(self.X[s], U, n)

    def core_term(self, s, U):
        return core_data_term(self.X[s], U)

    def dense(self, s):
        return self.X[s]


class TuckerData:
    """Compressed blocks X~^(s) = G^(s) x_1 A_1 x_2 A_2 x_3 A_3 with orthonormal
    A_n.  The two data terms use the Tucker form of eq. eqlrag / eqlrau:
    with W_m = A_m^T U^(m),

        M_(n) U^{⊙-n}   = A_n G_(n) W^{⊙-n}
        (U^⊙)^T vec(M)  = (W^⊙)^T vec(G)

    The paper's own Kruskal compression is the special case G = super-diagonal
    ones, A_n = U~^(n) (not orthonormal; then the identities still hold)."""

    def __init__(self, cores, factors):
        self.G = [np.asarray(g, dtype=np.float64) for g in cores]
        self.A = [[np.asarray(a, dtype=np.float64) for a in per_block] for per_block in factors]
        self._dense = [None] * len(self.G)

    @property
    def S(self):
        return len(self.G)

    def shape(self, s):
        return tuple(a.shape[0] for a in self.A[s])

    def _W(self, s, U):
        return [self.A[s][m].T @ U[m] for m in range(len(U))]

    def mttkrp(self, s, U, n):
        W = self._W(s, U)
        return self.A[s][n] @ (unfold(self.G[s], n) @ krp_minus(W, n))

    def core_term(self, s, U):
        W = self._W(s, U)
        return krp_all(W).T @ vec(self.G[s])

    def dense(self, s):
        if self._dense[s] is None:
            X = self.G[s]
            for n in range(X.ndim):
                X = mode_product(X, self.A[s][n], n)
            self._dense[s] = X
        return self._dense[s]


def objective(data, lam, U) -> float:
    """F = 1/2 sum_s ||M^(s) - [[D^(s); U^(1,s), ..., U^(N,s)]]||_F^2  (eq. costfunc),
    evaluated directly from the reconstruction."""
    total = 0.0
    for s in range(data.S):
        Us = [U[n][s] for n in range(len(U))]
        r = data.dense(s) - reconstruct(lam[s], Us)
        total += 0.5 * float(np.sum(r * r))
    return total


def block_relerrs(data, lam, U):
    out = []
    for s in range(data.S):
        Us = [U[n][s] for n in range(len(U))]
        X = data.dense(s)
        out.append(float(np.linalg.norm(X - reconstruct(lam[s], Us)) / np.linalg.norm(X)))
    return out


def relerr(data, lam, U) -> float:
    """RelErr = 1/S sum_s ||M - M^||_F / ||M||_F  (Section III-C, termination)."""
    return float(np.mean(block_relerrs(data, lam, U)))


def fit(tensors, lam, U) -> float:
    """Fit = 1/S sum_s (1 - ||M - M^||_F / ||M||_F)  (Section IV settings)."""
    return 1.0 - relerr(DenseData(tensors), lam, U)


# ---------------------------------------------------------------------------
# Algorithm 1 / 2
# ---------------------------------------------------------------------------


@dataclass
class Options:
    L: tuple                      # coupled columns per mode (first L_n columns shared)
    delta_w: float = 0.9999       # Appendix A
    tol: float = 1e-8             # Section III-C
    max_it: int = 1000
    restart: bool = True
    update_core: bool = True      # False: the -NC variant (D kept at its initial value)
    reset_t: bool = False
    # flexible coupling (Section III-C): per mode, the blocks that share the
    # first L_n columns (None: every block); the others keep all R columns
    # individual in that mode
    coupled_blocks: Optional[tuple] = None

    def group(self, n: int, S: int):
        """Blocks sharing mode n's first L_n columns, in block order."""
        if self.L[n] == 0:
            return []
        if self.coupled_blocks is None or self.coupled_blocks[n] is None:
            return list(range(S))
        return sorted(int(b) for b in self.coupled_blocks[n])


@dataclass
class State:
    U: List[List[np.ndarray]]        # [n][s], I_n x R, shared columns identical
    lam: List[np.ndarray]            # [s], R
    U_prev: List[List[np.ndarray]]   # x_{k-2}
    lam_prev: List[np.ndarray]
    Ld_prev: List[Optional[float]]   # [s]
    Lu_prev: List[List[Optional[float]]]  # [n][s]
    LC_prev: List[Optional[float]]   # [n]
    t: float = 1.0                   # t_{k-1}
    k: int = 0
    F: float = np.inf                # F_{k-1}
    relerr: float = np.inf
    restarts: int = 0
    history: list = field(default_factory=list)


def initial_state(data, U0, lam0) -> State:
    N = len(U0)
    S = len(lam0)
    U = [[np.array(U0[n][s], dtype=np.float64) for s in range(S)] for n in range(N)]
    lam = [np.array(l, dtype=np.float64) for l in lam0]
    st = State(U=U, lam=lam,
               U_prev=[[u.copy() for u in per] for per in U],
               lam_prev=[l.copy() for l in lam],
               Ld_prev=[None] * S, Lu_prev=[[None] * S for _ in range(N)], LC_prev=[None] * N)
    st.F = objective(data, st.lam, st.U)
    st.relerr = relerr(data, st.lam, st.U)
    return st


@dataclass
class SweepRecord:
    Ld: list
    Lu: list
    LC: list
    grads: dict = field(default_factory=dict)


def sweep(data, st: State, w_hat: float, extrapolate: bool, opt: Options):
    """One pass over every block in the paper's order.  Returns the new
    (lam, U) and the Lipschitz constants used."""
    N, S = len(st.U), len(st.lam)
    U = [[u.copy() for u in per] for per in st.U]
    lam = [l.copy() for l in st.lam]
    rec = SweepRecord(Ld=[None] * S, Lu=[[None] * S for _ in range(N)], LC=[None] * N)

    # (i) core tensors, eq. solD with the gradient of eq. solapgG and the
    #     extrapolated point of eq. eqextraPG
    for s in range(S):
        Us = [U[n][s] for n in range(N)]
        H = hadamard_of_grams(Us)
        Ld = spectral_norm(H)
        rec.Ld[s] = Ld
        if not opt.update_core or Ld <= 0.0:
            continue
        w = extrapolation_weight(w_hat, st.Ld_prev[s], Ld, opt.delta_w) if extrapolate else 0.0
        lam_hat = st.lam[s] + w * (st.lam[s] - st.lam_prev[s])
        G = H @ lam_hat - data.core_term(s, Us)
        lam[s] = np.maximum(0.0, lam_hat - G / Ld)
        rec.grads[("lam", s)] = G

    # (ii) factor matrices, eq. solUns / solUnC / solUnsI with the gradient of
    #      eq. solapgU and the extrapolated point of eq. eqextraPU
    for n in range(N):
        grp = opt.group(n, S)
        Ln = opt.L[n] if grp else 0
        P, Lu, K = [], [], []
        for s in range(S):
            Us = [U[m][s] for m in range(N)]
            Ps = np.outer(lam[s], lam[s]) * hadamard_of_grams(Us, skip=n)   # D H_{-n} D
            P.append(Ps)
            Lu.append(spectral_norm(Ps))
            K.append(data.mttkrp(s, Us, n))
        rec.Lu[n] = list(Lu)
        LC = float(sum(Lu[s] for s in grp)) if grp else float(sum(Lu))
        rec.LC[n] = LC

        Uhat = []
        for s in range(S):
            w = extrapolation_weight(w_hat, st.Lu_prev[n][s], Lu[s], opt.delta_w) if extrapolate else 0.0
            Uhat.append(st.U[n][s] + w * (st.U[n][s] - st.U_prev[n][s]))
        if Ln > 0:
            wC = extrapolation_weight(w_hat, st.LC_prev[n], LC, opt.delta_w) if extrapolate else 0.0
            g0 = grp[0]
            UC_old, UC_prev = st.U[n][g0][:, :Ln], st.U_prev[n][g0][:, :Ln]
            UC_hat = UC_old + wC * (UC_old - UC_prev)
            for s in grp:
                Uhat[s][:, :Ln] = UC_hat

        G = [Uhat[s] @ P[s] - K[s] * lam[s][None, :] for s in range(S)]
        for s in range(S):
            rec.grads[("U", n, s)] = G[s]

        if Ln > 0:
            if LC > 0.0:
                GC = sum(G[s][:, :Ln] for s in grp)
                UC_new = np.maximum(0.0, UC_hat - GC / LC)
            else:
                UC_new = st.U[n][grp[0]][:, :Ln].copy()
        for s in range(S):
            Ls = Ln if s in grp else 0          # blocks outside the group: all columns individual
            if Lu[s] > 0.0:
                UI_new = np.maximum(0.0, Uhat[s][:, Ls:] - G[s][:, Ls:] / Lu[s])
            else:
                UI_new = st.U[n][s][:, Ls:].copy()
            U[n][s] = np.concatenate([UC_new, UI_new], axis=1) if Ls > 0 else UI_new
    return lam, U, rec


def iterate(data, st: State, opt: Options) -> State:
    """One accepted outer iteration k of Algorithm 1 (restart included)."""
    t_k = t_next(st.t)
    w_hat = (st.t - 1.0) / t_k
    lam, U, rec = sweep(data, st, w_hat, True, opt)
    F = objective(data, lam, U)
    restarted = False
    if opt.restart and F >= st.F:
        lam, U, rec = sweep(data, st, w_hat, False, opt)
        F = objective(data, lam, U)
        restarted = True
    new = State(U=U, lam=lam, U_prev=st.U, lam_prev=st.lam,
                Ld_prev=list(rec.Ld), Lu_prev=[list(x) for x in rec.Lu], LC_prev=list(rec.LC),
                t=(1.0 if (restarted and opt.reset_t) else t_k), k=st.k + 1, F=F,
                relerr=relerr(data, lam, U), restarts=st.restarts + int(restarted),
                history=st.history + [(st.k + 1, F, restarted)])
    new.last_record = rec
    new.last_restarted = restarted
    return new


def run(data, U0, lam0, opt: Options, iters: Optional[int] = None, state: Optional[State] = None) -> State:
    """Algorithm 1 (dense data) or the iteration part of Algorithm 2 (Tucker data).
    Stops after ``iters`` iterations if given, else at |dRelErr| < tol or max_it."""
    st = state if state is not None else initial_state(data, U0, lam0)
    limit = iters if iters is not None else opt.max_it
    for _ in range(limit):
        prev_rel = st.relerr
        st = iterate(data, st, opt)
        if iters is None and abs(st.relerr - prev_rel) < opt.tol:
            break
    return st


# ---------------------------------------------------------------------------
# Loss and block gradients at one point (all blocks at the same point)
# ---------------------------------------------------------------------------


def loss_and_grads(data, lam, U, L, coupled_blocks=None):
    """F and its partial gradients at (lam, U): d/dlam^(s) = H lam - b
    (eq. solbpgG) and d/dU^(n,s) = U D H_{-n} D - M_(n) U^{⊙-n} D
    (eq. solbpgU).  The shared columns' gradient is the sum over s
    (eq. solbpgUCI summed over the blocks that share U_C)."""
    N, S = len(U), len(lam)
    F = objective(data, lam, U)
    g_lam, g_U = [], [[None] * S for _ in range(N)]
    for s in range(S):
        Us = [U[n][s] for n in range(N)]
        g_lam.append(hadamard_of_grams(Us) @ lam[s] - data.core_term(s, Us))
        for n in range(N):
            P = np.outer(lam[s], lam[s]) * hadamard_of_grams(Us, skip=n)
            g_U[n][s] = U[n][s] @ P - data.mttkrp(s, Us, n) * lam[s][None, :]
    g_C = []
    grp = Options(L=tuple(L), coupled_blocks=coupled_blocks)
    for n in range(N):
        Ln = L[n]
        g_C.append(sum(g_U[n][s][:, :Ln] for s in grp.group(n, S)) if Ln > 0 else None)
    return F, g_lam, g_U, g_C
