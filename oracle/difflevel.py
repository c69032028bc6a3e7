"""Difference levels of MGMLMC: exact deflation of each difference operator (Sec. 4.2,
eqs. 15-16) and the split that skips a level (Sec. 4.1, eq. 12) (oracle; test only).

A term of the telescoping sum joins hierarchy level a to a coarser level b; with the
composite interpolation P_ab = P_a P_{a+1} ... P_{b-1} its operator is

    M_ab = D_a^-1 - P_ab D_b^-1 P_ab^H.

b = a + 1 is the term of eq. 11; b = a + 2 skips level a + 1 (eq. 12 skips level 2 of a
four-level hierarchy: terms (1, 3), (3, 4) and the coarsest term of level 4).

Deflation (Sec. 4.2).  Gamma5 commutes with every P_l (eq. 14), hence with P_ab, and
Q_l = Gamma5 D_l is Hermitian, so J_ab = M_ab Gamma5 = Q_a^-1 - P_ab Q_b^-1 P_ab^H is
Hermitian (eq. 15).  From J_ab = X Lambda X^H (eq. 16): M_ab = X Lambda X^H Gamma5 with left
singular vectors U = X sign(Lambda), singular values |Lambda| and right singular vectors
V = Gamma5 X.  The k eigenpairs of largest |lambda| (ties: lambda descending) give the k
largest singular triplets; with Pi = V V^H

    tr(M_ab) = tr(M_ab (I - Pi)) + tr(M_ab Pi),   tr(M_ab Pi) = sum_i lambda_i x_i^H Gamma5 x_i,

because M_ab v_i = X Lambda X^H x_i = lambda_i x_i.  A deflated sample of the term is
s = x^H M_ab (x - V V^H x) = x^H D_a^-1 xt - y^H D_b^-1 yt with xt = x - V V^H x,
y = P_ab^H x, yt = P_ab^H xt; x is the real Z2 vector of sample i of level a.

Inexact deflation (Sec. 3.2 for D; here for M_ab): with approximate eigenvectors X (any
orthonormal k columns) the split still holds with Pi = V V^H, V = Gamma5 X, but the small
term must be evaluated, tr(M_ab Pi) = sum_i v_i^H M_ab v_i = sum_i x_i^H Gamma5 J_ab x_i,
at the price of k extra applications of J (the "k extra inversions" of the text); its real
part enters the estimate.

Eigensolvers: dense numpy.linalg.eigh of J (small levels) or scipy's ARPACK (eigsh,
largest magnitude) on J as a linear operator whose solves are sparse LU.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import noise
from .mlmc import DirectSolver


def composite_P(levels, a: int, b: int) -> sp.csr_matrix:
    """P_a P_{a+1} ... P_{b-1}: level b -> level a (1-based, a < b)."""
    P = levels[a - 1].P.tocsr()
    for l in range(a + 1, b):
        P = P @ levels[l - 1].P
    return P.tocsr()


def terms(L: int, skip: Sequence[int] = ()) -> List[Tuple[int, int]]:
    """Difference terms (a, b) of the telescoping sum over the levels not in `skip`."""
    keep = [l for l in range(1, L + 1) if l not in set(skip)]
    if keep[0] != 1 or keep[-1] != L:
        raise ValueError("the finest and the coarsest level cannot be skipped")
    return list(zip(keep[:-1], keep[1:]))


def J_dense(levels, a: int, b: int) -> np.ndarray:
    """J_ab = Q_a^-1 - P_ab Q_b^-1 P_ab^H, dense (small levels)."""
    Qa = (levels[a - 1].gamma5 @ levels[a - 1].D).toarray()
    Qb = (levels[b - 1].gamma5 @ levels[b - 1].D).toarray()
    P = composite_P(levels, a, b).toarray()
    return np.linalg.inv(Qa) - P @ np.linalg.inv(Qb) @ P.conj().T


def M_dense(levels, a: int, b: int) -> np.ndarray:
    """M_ab = D_a^-1 - P_ab D_b^-1 P_ab^H, dense (small levels)."""
    P = composite_P(levels, a, b).toarray()
    return (np.linalg.inv(levels[a - 1].D.toarray())
            - P @ np.linalg.inv(levels[b - 1].D.toarray()) @ P.conj().T)


def J_operator(levels, solver: DirectSolver, a: int, b: int) -> spla.LinearOperator:
    """J_ab as a linear operator: Q^-1 v = D^-1 Gamma5 v by sparse LU."""
    P = composite_P(levels, a, b)
    g5a = levels[a - 1].gamma5
    g5b = levels[b - 1].gamma5
    n = levels[a - 1].n

    def mv(v):
        v = np.asarray(v, dtype=np.complex128).reshape(n, -1)
        out = solver.solve(a, g5a @ v) - P @ solver.solve(b, g5b @ (P.conj().T @ v))
        return out if out.shape[1] > 1 else out[:, 0]

    return spla.LinearOperator((n, n), matvec=mv, matmat=mv, dtype=np.complex128)


def largest_eigenpairs(lam: np.ndarray, X: np.ndarray, k: int):
    order = np.lexsort((-lam, -np.abs(lam)))[:k]
    return lam[order], X[:, order]


@dataclass
class DiffDeflation:
    a: int
    b: int
    X: np.ndarray     # n_a x k eigenvectors of J_ab
    lam: np.ndarray   # k eigenvalues (signed, largest |lambda| first)
    V: np.ndarray     # Gamma5 X: right singular vectors of M_ab
    corr: float       # tr(M_ab Pi) = sum lambda_i x_i^H Gamma5 x_i (real: J Hermitian)


def deflate_difference(levels, a: int, b: int, k: int, method: str = "dense",
                       solver: Optional[DirectSolver] = None, tol: float = 1e-12) -> DiffDeflation:
    if method == "dense":
        lam, X = np.linalg.eigh(J_dense(levels, a, b))
        lam, X = largest_eigenpairs(lam, X, k)
    elif method == "arpack":
        solver = solver or DirectSolver(levels)
        lam, X = spla.eigsh(J_operator(levels, solver, a, b), k=k, which="LM", tol=tol)
        lam, X = largest_eigenpairs(lam, X, k)
    else:
        raise ValueError(method)
    g5 = levels[a - 1].gamma5
    V = np.asarray(g5 @ X)
    corr = float(np.real(np.sum(lam * np.einsum("ik,ik->k", X.conj(), V))))
    return DiffDeflation(a=a, b=b, X=X, lam=lam, V=V, corr=corr)


def pair_terms(levels, solver: DirectSolver, a: int, b: int, x: np.ndarray,
               dd: Optional[DiffDeflation] = None):
    """(x^H D_a^-1 xt, y^H D_b^-1 yt) with xt = x - V V^H x (x when dd is None),
    y = P_ab^H x, yt = P_ab^H xt; x may hold one noise vector per column."""
    xt = x if dd is None else x - dd.V @ (dd.V.conj().T @ x)
    P = composite_P(levels, a, b)
    y = P.conj().T @ x
    yt = P.conj().T @ xt
    return (np.sum(x.conj() * solver.solve(a, xt), axis=0),
            np.sum(y.conj() * solver.solve(b, yt), axis=0))


def pair_sample(levels, solver: DirectSolver, seed: int, a: int, b: int, i: int,
                dd: Optional[DiffDeflation] = None):
    """(s, t1, t2) for sample i of term (a, b); the noise is that of level a."""
    x = noise.z2_noise(seed, a, i, levels[a - 1].n)
    t1, t2 = pair_terms(levels, solver, a, b, x, dd)
    return complex(t1 - t2), complex(t1), complex(t2)


def inexact_deflation(levels, a: int, b: int, X: np.ndarray, solver: Optional[DirectSolver] = None,
                      dense: bool = False) -> DiffDeflation:
    """Deflation of term (a, b) by given orthonormal columns X: lam are the Rayleigh quotients
    x_i^H J x_i, corr = Re sum_i x_i^H Gamma5 J x_i (k applications of J)."""
    if dense:
        JX = J_dense(levels, a, b) @ X
    else:
        JX = J_operator(levels, solver or DirectSolver(levels), a, b).matmat(X)
    g5 = levels[a - 1].gamma5
    V = np.asarray(g5 @ X)
    lam = np.real(np.einsum("ik,ik->k", X.conj(), JX))
    corr = float(np.real(np.sum(np.einsum("ik,ik->k", V.conj(), JX))))
    return DiffDeflation(a=a, b=b, X=X, lam=lam, V=V, corr=corr)
