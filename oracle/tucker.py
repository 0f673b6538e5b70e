"""FP64 CPU oracle for the compression step of lraCoNCPD-APG.

TEST INFRASTRUCTURE (see the header of ``oracle.apg``).

The paper compresses each block before the iterations (Algorithm 2, first
step; Section III-B).  The workloads here compress with a truncated
higher-order SVD (De Lathauwer, De Moor, Vandewalle 2000): the mode-n basis
A_n holds the J_n leading left singular vectors of M_(n), i.e. the leading
eigenvectors of M_(n) M_(n)^T, and the core is G = M x_1 A_1^T x_2 A_2^T
x_3 A_3^T.  Every Gram is taken from the original tensor (not sequentially
truncated).  Eigenvectors come in descending eigenvalue order; each is signed
so that its entry of largest magnitude is positive.
"""
from __future__ import annotations

import numpy as np

from .apg import mode_product, unfold


def leading_eigvecs(S: np.ndarray, J: int):
    """The J leading eigenpairs of a symmetric PSD matrix (numpy.linalg.eigh),
    descending, with the sign convention above."""
    evals, evecs = np.linalg.eigh(S)
    order = np.argsort(evals)[::-1][:J]
    A = evecs[:, order].copy()
    for j in range(A.shape[1]):
        k = int(np.argmax(np.abs(A[:, j])))
        if A[k, j] < 0:
            A[:, j] = -A[:, j]
    return evals[order], A


def thosvd(X: np.ndarray, ranks):
    """Truncated HOSVD of a 3-way tensor.  Returns (G, [A_1, A_2, A_3], eigenvalues)."""
    X = np.asarray(X, dtype=np.float64)
    A, ev = [], []
    for n in range(X.ndim):
        Xn = unfold(X, n)
        e, An = leading_eigvecs(Xn @ Xn.T, ranks[n])
        A.append(An)
        ev.append(e)
    G = X
    for n in range(X.ndim):
        G = mode_product(G, A[n].T, n)
    return G, A, ev


def compress_all(tensors, ranks):
    """T-HOSVD of every block: lists of cores, bases and Gram eigenvalues."""
    cores, bases, evs = [], [], []
    for X in tensors:
        G, A, e = thosvd(X, ranks)
        cores.append(G)
        bases.append(A)
        evs.append(e)
    return cores, bases, evs
