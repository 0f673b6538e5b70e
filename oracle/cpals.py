"""FP64 CPU oracle for the paper's own compression step of lraCoNCPD-APG:
an unconstrained CPD of every block fitted by alternating least squares.

TEST INFRASTRUCTURE (see the header of ``oracle.apg``).

Algorithm 2 first approximates each block by a rank-R~ unconstrained CPD
(Section III-B, eq. cosfunclra) and the experiment settings (Section IV) fit
it by ALS, stopping once the relative error changes by less than 1e-4 or
after 200 iterations.  One ALS iteration updates U~^(1), U~^(2), U~^(3) in
turn, each as the exact least-squares solution with the other two fixed:

    U~^(n) = M_(n) U~^{⊙-n} (⊛_{m≠n} U~^(m)T U~^(m))^{-1}

(normal equations of min ||M_(n) - U~^(n) (U~^{⊙-n})^T||_F).  The compressed
block is X~ = [[U~^(1), U~^(2), U~^(3)]], the Tucker form with a super-diagonal
core of ones.

Readings of points the paper leaves open (also listed in the design notes):

* The starting point is an input (the library draws it U[0,1] when the caller
  gives none).
* RelErr_0 is taken at the starting point; the stopping test after iteration
  k compares RelErr_k with RelErr_{k-1}, as the paper's rule for the coupled
  algorithms does.
* No column normalisation between the updates (the fitted model is the same
  in exact arithmetic; the scaling is absorbed by the next update).
* Every block is fitted and stopped on its own.
"""
from __future__ import annotations

import numpy as np

from .apg import hadamard_of_grams, mttkrp, reconstruct


def relerr(X: np.ndarray, U) -> float:
    """||X - [[U]]||_F / ||X||_F by explicit reconstruction."""
    Xh = reconstruct(np.ones(U[0].shape[1]), U)
    return float(np.linalg.norm(X - Xh) / np.linalg.norm(X))


def als_iteration(X: np.ndarray, U):
    """One ALS iteration (modes in order, each using the latest others)."""
    U = [np.array(u, dtype=np.float64) for u in U]
    for n in range(X.ndim):
        V = hadamard_of_grams(U, skip=n)
        K = mttkrp(X, U, n)
        U[n] = np.linalg.solve(V, K.T).T     # K V^{-1}; V is symmetric
    return U


def cp_als(X: np.ndarray, U0, eps: float = 1e-4, max_it: int = 200):
    """Fit [[U~]] to X.  Returns (U~, iterations run, RelErr history starting
    with RelErr_0)."""
    X = np.asarray(X, dtype=np.float64)
    U = [np.array(u, dtype=np.float64) for u in U0]
    hist = [relerr(X, U)]
    it = 0
    while it < max_it:
        U = als_iteration(X, U)
        it += 1
        hist.append(relerr(X, U))
        if abs(hist[-1] - hist[-2]) < eps:
            break
    return U, it, hist


def compress_all_cp(tensors, inits, eps: float = 1e-4, max_it: int = 200):
    """CP-ALS of every block: factor lists, iteration counts, final RelErr."""
    facs, its, rels = [], [], []
    for X, U0 in zip(tensors, inits):
        U, it, hist = cp_als(X, U0, eps, max_it)
        facs.append(U)
        its.append(it)
        rels.append(hist[-1])
    return facs, its, rels


def kruskal_as_tucker(U):
    """(core, bases) of [[U]] in Tucker form: super-diagonal ones, A_n = U_n."""
    R = U[0].shape[1]
    G = np.zeros((R,) * len(U))
    for r in range(R):
        G[(r,) * len(U)] = 1.0
    return G, [np.array(u, dtype=np.float64) for u in U]
