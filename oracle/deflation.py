"""Exact deflation of the coarsest operator from the eigenpairs of Q = Gamma5 D (oracle; test only).

Sec. 2: Pi = U_k U_k^H with U_k the k smallest left singular vectors of D (eq. 4); the
trace splits as tr(D^-1 (I - Pi)) + tr(D^-1 Pi) (eq. 5); the small term is
tr(U_k^H V_k Sigma_k^-1) (eq. 6).  With Q = Gamma5 D Hermitian and Q = X Lambda X^H
(eq. 7): U = Gamma5 X sign(Lambda), V = X, Sigma = |Lambda|.  Hence

    Pi = W W^H with W = Gamma5 X_k   (the sign drops out),
    tr(D^-1 Pi) = sum_i (x_i^H Gamma5 x_i) / lambda_i.

The k eigenpairs with the smallest |lambda| are taken, ties broken by lambda ascending.
Dense numpy.linalg.eigh is the eigensolver.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Deflation:
    W: np.ndarray        # n x k, columns Gamma5 x_i
    X: np.ndarray        # n x k eigenvectors of Q
    lam: np.ndarray      # k eigenvalues of Q (signed)
    tr_defl: float       # tr(D^-1 Pi)


def smallest_eigenpairs(Q: np.ndarray, k: int):
    lam, X = np.linalg.eigh(Q)
    order = np.lexsort((lam, np.abs(lam)))[:k]
    return lam[order], X[:, order]


def deflate(D: sp.spmatrix, gamma5: sp.spmatrix, k: int) -> Deflation:
    Q = (gamma5 @ D).toarray()
    lam, X = smallest_eigenpairs(Q, k)
    W = gamma5 @ X
    g5 = gamma5.diagonal().real
    tr = float(np.sum(np.einsum("ik,i,ik->k", X.conj(), g5, X).real / lam))
    return Deflation(W=np.asarray(W), X=X, lam=lam, tr_defl=tr)


def project_out(W: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(I - W W^H) x."""
    return x - W @ (W.conj().T @ x)
