"""Solvers of the checker for level operators too large for a plain sparse LU (oracle; test only).

The checker's sample values need x^H D_l^-1 x at every level (eq. 11).  Up to a few
hundred thousand unknowns a sparse LU does this directly.  The 1024^2 workload has a
fine operator with 2M unknowns and a level-2 operator with 1M unknowns in dense 16 x 16
blocks (SuperLU cannot hold the latter's factors), so two more solvers are provided:

* ``NDLU``: sparse LU of D after a symmetric permutation that orders the lattice sites
  by geometric nested dissection (a permutation changes the fill, not the solution;
  rows are still exchanged where a pivot is below 0.1 of its column),
  followed by iterative refinement with the unpermuted operator until the relative
  residual stops decreasing;
* ``fgmres`` with a ``VCycle`` preconditioner: flexible GMRES (Saad, SIAM J. Sci. Comput.
  14, 1993), right-preconditioned by the multigrid iteration of Sec. 3.1, eq. (8),
  applied recursively down the hierarchy with block-Jacobi smoothing (one of the
  smoothers the paper names) and a sparse LU at the level where the recursion stops.

Every result of these solvers is a vector x with a stated relative residual
||b - D x|| / ||b||, recomputed with the operator itself; that residual is what pins them
(and ``HybridSolver.solve`` raises if it is not met).
"""
from __future__ import annotations

import time
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mass import nested_dissection_sites
from .multigrid import Level


def relres(D: sp.spmatrix, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """||b - D x|| / ||b|| per column (or for one vector)."""
    r = b - D @ x
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)


class NDLU:
    """Sparse LU of a level operator in nested-dissection site order, with refinement."""

    def __init__(self, level: Level):
        self.D = level.D.tocsr()
        s = nested_dissection_sites(level.Lx, level.Lt)
        d = level.dofs
        self.p = (d * s[:, None] + np.arange(d)[None, :]).ravel()
        Dp = self.D[self.p][:, self.p].tocsc()
        self.lu = spla.splu(Dp, permc_spec="NATURAL", diag_pivot_thresh=0.1)

    def _solve_once(self, b: np.ndarray) -> np.ndarray:
        y = self.lu.solve(np.ascontiguousarray(b[self.p]))
        x = np.empty_like(y)
        x[self.p] = y
        return x

    def solve(self, b: np.ndarray, max_refine: int = 5) -> np.ndarray:
        b = np.asarray(b, dtype=np.complex128)
        x = self._solve_once(b)
        res = np.max(relres(self.D, x, b))
        for _ in range(max_refine):
            x_new = x + self._solve_once(b - self.D @ x)
            res_new = np.max(relres(self.D, x_new, b))
            if not res_new < res:
                break
            x, res = x_new, res_new
        return x


class BlockJacobi:
    """x <- x + omega B^-1 (b - D x) with B the d x d self blocks of the sites (a level with
    d dofs per site)."""

    def __init__(self, level: Level, omega: float):
        d = level.dofs
        ns = level.Lx * level.Lt
        D = level.D.tocsr()
        coo = D.tocoo()
        own = coo.row // d == coo.col // d
        blocks = np.zeros((ns, d, d), dtype=np.complex128)
        blocks[coo.row[own] // d, coo.row[own] % d, coo.col[own] % d] = coo.data[own]
        self.Binv = np.linalg.inv(blocks)
        self.D = D
        self.d = d
        self.omega = omega

    def apply_inverse_blocks(self, r: np.ndarray) -> np.ndarray:
        rs = r.reshape(-1, self.d)
        return np.einsum("sij,sj->si", self.Binv, rs).reshape(-1)

    def sweeps(self, b: np.ndarray, x: np.ndarray, nu: int) -> np.ndarray:
        for _ in range(nu):
            x = x + self.omega * self.apply_inverse_blocks(b - self.D @ x)
        return x


class VCycle:
    """The multigrid iteration of eq. (8), recursive from level `top` down to level
    `bottom`, where D_bottom^-1 is a sparse LU; smoother S = nu block-Jacobi sweeps."""

    def __init__(self, levels: Sequence[Level], top: int, bottom: int, nu_pre: int = 1, nu_post: int = 2,
                 omega: float = 0.8):
        if not 1 <= top < bottom <= len(levels):
            raise ValueError("need top < bottom within the hierarchy")
        self.levels = levels
        self.top, self.bottom = top, bottom
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.smooth = {l: BlockJacobi(levels[l - 1], omega) for l in range(top, bottom)}
        self.coarse = NDLU(levels[bottom - 1])

    def apply(self, b: np.ndarray, l: Optional[int] = None) -> np.ndarray:
        """Approximates D_l^-1 b by one iteration of eq. (8) from x = 0."""
        l = self.top if l is None else l
        if l == self.bottom:
            return self.coarse.solve(b)
        lv = self.levels[l - 1]
        S = self.smooth[l]
        x = S.sweeps(b, np.zeros_like(b), self.nu_pre)
        r = b - lv.D @ x
        x = x + lv.P @ self.apply(lv.P.conj().T @ r, l + 1)
        return S.sweeps(b, x, self.nu_post)


def fgmres(matvec: Callable[[np.ndarray], np.ndarray], b: np.ndarray,
           precond: Callable[[np.ndarray], np.ndarray], rtol: float, restart: int = 40,
           max_cycles: int = 100):
    """Right-preconditioned flexible GMRES(restart) for one vector b, from x = 0.

    Each cycle builds the Arnoldi relation A Z_m = V_{m+1} H_m with z_j = precond(v_j),
    orthogonalising by modified Gram-Schmidt done twice, and takes the minimiser y of
    ||beta e_1 - H_m y|| (numpy least squares); x += Z_m y.  The cycle ends when that
    least-squares residual is below rtol/2 relative to ||b||; the solve ends when the
    residual b - A x recomputed from x is below rtol.  Returns (x, relres, iterations).
    """
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, 0.0, 0
    iters = 0
    for _ in range(max_cycles):
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm:
            return x, beta / bnorm, iters
        V: List[np.ndarray] = [r / beta]
        Z: List[np.ndarray] = []
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        y = np.zeros(0, dtype=np.complex128)
        for j in range(restart):
            Z.append(precond(V[j]))
            w = matvec(Z[j])
            for _pass in range(2):
                for i in range(j + 1):
                    h = np.vdot(V[i], w)
                    H[i, j] += h
                    w = w - h * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            iters += 1
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
            est = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
            if est <= 0.5 * rtol * bnorm or H[j + 1, j] == 0.0:
                break
            V.append(w / H[j + 1, j])
        x = x + np.column_stack(Z[:y.size]) @ y
    r = b - matvec(x)
    return x, np.linalg.norm(r) / bnorm, iters


class HybridSolver:
    """D_l^-1 b for every level of a hierarchy, as oracle.mlmc.DirectSolver does, choosing
    per level: the ND-ordered sparse LU for the fine Wilson level and for levels with
    n <= lu_max, else FGMRES preconditioned by the V-cycle of eq. (8) from that level down
    to the first level with n <= lu_max.  Columns of b are solved one after another
    (iteratively) or together (LU); every solve must reach rtol (recomputed residual) or
    this raises."""

    def __init__(self, levels: Sequence[Level], rtol: float = 1e-13, lu_max: int = 70000, restart: int = 40,
                 log: Optional[Callable[[str], None]] = None):
        self.levels = levels
        self.rtol = rtol
        self.lu_max = lu_max
        self.restart = restart
        self.log = log
        self._lu = {}
        self._mg = {}
        self.iterations = {}

    def uses_lu(self, l: int) -> bool:
        lv = self.levels[l - 1]
        return lv.n <= self.lu_max or l == 1

    def prepare(self, l: int):
        """Builds what level l's solves need (its LU, or its V-cycle with its smoothers and
        the LU at the bottom), once."""
        t = time.time()
        if self.uses_lu(l):
            if l in self._lu:
                return
            self._lu[l] = NDLU(self.levels[l - 1])
            what = "LU"
        else:
            if l in self._mg:
                return
            bottom = next(j for j in range(l + 1, len(self.levels) + 1) if self.levels[j - 1].n <= self.lu_max)
            self._mg[l] = VCycle(self.levels, l, bottom)
            what = f"V-cycle down to level {bottom}"
        if self.log:
            self.log(f"level {l}: {what} for n = {self.levels[l - 1].n} in {time.time() - t:.1f} s")

    def solve(self, l: int, b: np.ndarray) -> np.ndarray:
        b = np.asarray(b, dtype=np.complex128)
        self.prepare(l)
        D = self.levels[l - 1].D
        if self.uses_lu(l):
            x = self._lu[l].solve(b)
            res = np.max(relres(D, x, b))
            if not res <= self.rtol:
                raise RuntimeError(f"LU solve at level {l} left relative residual {res:.3g} > {self.rtol:.1e}")
            return x
        cols = b.reshape(b.shape[0], -1)
        out = np.empty_like(cols)
        for c in range(cols.shape[1]):
            t = time.time()
            x, res, it = fgmres(lambda v: D @ v, cols[:, c], self._mg[l].apply, self.rtol, self.restart)
            if not res <= self.rtol:
                raise RuntimeError(f"FGMRES at level {l} stopped at relative residual {res:.3g} > {self.rtol:.1e}")
            self.iterations.setdefault(l, []).append(it)
            if self.log:
                self.log(f"level {l}: FGMRES {it} iterations, relres {res:.2e}, {time.time() - t:.1f} s")
            out[:, c] = x
        return out.reshape(b.shape)
