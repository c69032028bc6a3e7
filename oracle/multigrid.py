"""Aggregation multigrid hierarchy: test vectors, interpolator P, Galerkin D_{l+1} = P^H D_l P.

(oracle; test only)

The paper's two-level iteration and Petrov-Galerkin coarse operator are Sec. 3.1, eq. (8)
and the sentence after it (R_l = P_l^H, P_l^H P_l = I as noted before eq. 11); the
aggregation construction is cited, not given (Sec. 3.1, last paragraph), and the
"spin-preserving" relations it must satisfy are eq. (14).  Readings used here:

* Aggregates are ax x at blocks of sites of the level-l lattice, tiled lexicographically;
  aggregate (X, T) is coarse site X + Lx_{l+1} * T.
* N test vectors per chirality: each full test vector is split by chirality on every
  aggregate, so a coarse site has 2N dofs ordered [chirality +: tv 0..N-1,
  chirality -: tv 0..N-1] and the coarse Gamma5 is diag(+1 x N, -1 x N).  At a coarse
  level, chirality + is the first half of a site's dofs.
* On each (aggregate, chirality) block the test vectors are orthonormalised by modified
  Gram-Schmidt in column order, which is the QR factorisation with a positive real
  diagonal of R; the Q factor is that block of P.  This makes P unique and P^H P = I.
* Test vectors (parity unpinned: the paper cites its setup): V_0 = N Z4 start vectors;
  n_inv times V <- D_l^{-1} V (exact, direct LU solve), then V <- MGS(V) in column
  order.  Because MGS only right-multiplies V by an upper-triangular matrix with a
  positive diagonal, the final P equals the local QR of D_l^{-n_inv} V_0.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import noise, wilson


@dataclass
class Level:
    Lx: int
    Lt: int
    dofs: int
    D: sp.csr_matrix
    P: Optional[sp.csr_matrix] = None      # interpolation to this level from the next coarser
    V: Optional[np.ndarray] = None         # test vectors used to build P (n x N)
    agg: Optional[tuple] = None            # (ax, at) used to coarsen this level
    N: Optional[int] = None                # test vectors per chirality

    @property
    def n(self) -> int:
        return self.Lx * self.Lt * self.dofs

    @property
    def gamma5(self) -> sp.csr_matrix:
        return wilson.gamma5(self.Lx * self.Lt, self.dofs)


def chirality_dofs(dofs: int, c: int) -> np.ndarray:
    half = dofs // 2
    return np.arange(c * half, (c + 1) * half)


def aggregate_block_rows(Lx: int, Lt: int, dofs: int, ax: int, at: int, X: int, T: int, c: int):
    """Level-l row indices of aggregate (X, T), chirality c."""
    rows = []
    for t in range(T * at, (T + 1) * at):
        for x in range(X * ax, (X + 1) * ax):
            s = x + Lx * t
            for dof in chirality_dofs(dofs, c):
                rows.append(dofs * s + dof)
    return np.array(rows, dtype=np.int64)


def mgs(V: np.ndarray) -> np.ndarray:
    """Modified Gram-Schmidt in column order; columns of the result are orthonormal."""
    Q = np.array(V, dtype=np.complex128, copy=True)
    for k in range(Q.shape[1]):
        for j in range(k):
            Q[:, k] -= np.vdot(Q[:, j], Q[:, k]) * Q[:, j]
        nrm = np.linalg.norm(Q[:, k])
        if nrm == 0.0:
            raise ValueError("rank-deficient test vectors")
        Q[:, k] /= nrm
    return Q


def check_geometry(Lx: int, Lt: int, dofs: int, ax: int, at: int, N: int):
    if Lx % ax or Lt % at:
        raise ValueError(f"lattice {Lx}x{Lt} not divisible by aggregate {ax}x{at}")
    if Lx // ax < 2 or Lt // at < 2:
        raise ValueError("coarse lattice extent must be at least 2 in each direction")
    if ax * at * (dofs // 2) < N:
        raise ValueError("more test vectors than rows per aggregate and chirality")


def start_vectors(seed: int, level: int, N: int, n: int) -> np.ndarray:
    return np.column_stack([noise.z4_start(seed, level, v, n) for v in range(N)])


def test_vectors(D: sp.csr_matrix, N: int, n_inv: int, seed: int, level: int) -> np.ndarray:
    """V = MGS(D^-1 ... MGS(D^-1 V_0)) with exact (direct) solves."""
    n = D.shape[0]
    V = start_vectors(seed, level, N, n)
    lu = spla.splu(D.tocsc())
    for _ in range(n_inv):
        V = lu.solve(V)
        V = mgs(V)
    return V


def interpolator(V: np.ndarray, Lx: int, Lt: int, dofs: int, ax: int, at: int) -> sp.csr_matrix:
    """P (n_l x n_{l+1}) from test vectors V: per (aggregate, chirality) the Q factor of
    the QR factorisation with positive real diagonal (MGS)."""
    N = V.shape[1]
    Lxc, Ltc = Lx // ax, Lt // at
    n_f = Lx * Lt * dofs
    n_c = Lxc * Ltc * 2 * N
    rows, cols, vals = [], [], []
    for T in range(Ltc):
        for X in range(Lxc):
            cs = X + Lxc * T
            for c in range(2):
                r = aggregate_block_rows(Lx, Lt, dofs, ax, at, X, T, c)
                Q = mgs(V[r, :])
                for k in range(N):
                    rows.append(r)
                    cols.append(np.full(r.size, 2 * N * cs + c * N + k))
                    vals.append(Q[:, k])
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_f, n_c)).tocsr()
    return P


def galerkin(D: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """Petrov-Galerkin coarse operator R D P with R = P^H."""
    Dc = (P.conj().T @ D @ P).tocsr()
    Dc.sum_duplicates()
    return Dc


def build_hierarchy(theta: np.ndarray, m0: float, aggs, ntv, n_inv: int, seed: int,
                    import_tv: Optional[List[np.ndarray]] = None) -> List[Level]:
    """Levels 1..L: fine Wilson-Schwinger D, then P_l and D_{l+1} = P_l^H D_l P_l."""
    _, Lt, Lx = theta.shape
    levels = [Level(Lx, Lt, 2, wilson.dirac_operator(theta, m0))]
    for l, ((ax, at), N) in enumerate(zip(aggs, ntv)):
        cur = levels[-1]
        check_geometry(cur.Lx, cur.Lt, cur.dofs, ax, at, N)
        if import_tv is not None:
            V = np.asarray(import_tv[l], dtype=np.complex128)
        else:
            V = test_vectors(cur.D, N, n_inv, seed, l + 1)
        P = interpolator(V, cur.Lx, cur.Lt, cur.dofs, ax, at)
        cur.P, cur.V, cur.agg, cur.N = P, V, (ax, at), N
        levels.append(Level(cur.Lx // ax, cur.Lt // at, 2 * N, galerkin(cur.D, P)))
    return levels


DIRS = ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1))   # self, +x, -x, +t, -t


def coarse_blocks(Dc: sp.csr_matrix, Lx: int, Lt: int, dofs: int) -> np.ndarray:
    """Dense blocks A[site, dir] (dofs x dofs) of a nearest-neighbour block operator,
    dir in (self, +x, -x, +t, -t): (Dc psi)_s = sum_dir A[s, dir] psi_{s + dir}.

    Where a lattice extent is 2, s + mu and s - mu are one site: the whole coupling is
    stored in the +mu block and the -mu block is zero.  Raises if Dc couples sites that
    are not nearest neighbours.
    """
    ns = Lx * Lt
    A = np.zeros((ns, 5, dofs, dofs), dtype=np.complex128)
    Dc = Dc.tocsr()
    for t in range(Lt):
        for x in range(Lx):
            s = x + Lx * t
            rowblk = Dc[s * dofs:(s + 1) * dofs, :]
            seen = set()
            for d, (dx, dt) in enumerate(DIRS):
                nb = (x + dx) % Lx + Lx * ((t + dt) % Lt)
                if nb in seen:
                    continue
                seen.add(nb)
                A[s, d] = rowblk[:, nb * dofs:(nb + 1) * dofs].toarray()
    stray = abs(Dc - blocks_to_sparse(A, Lx, Lt)).max()
    if stray != 0.0:
        raise ValueError(f"operator is not a nearest-neighbour block stencil (stray {stray})")
    return A


def blocks_to_sparse(A: np.ndarray, Lx: int, Lt: int) -> sp.csr_matrix:
    """Inverse of coarse_blocks: the sparse operator of a block stencil."""
    ns, _, dofs, _ = A.shape
    rows, cols, vals = [], [], []
    base = np.arange(dofs)
    for t in range(Lt):
        for x in range(Lx):
            s = x + Lx * t
            for d, (dx, dt) in enumerate(DIRS):
                nb = (x + dx) % Lx + Lx * ((t + dt) % Lt)
                rr, cc = np.meshgrid(s * dofs + base, nb * dofs + base, indexing="ij")
                rows.append(rr.ravel())
                cols.append(cc.ravel())
                vals.append(A[s, d].ravel())
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(ns * dofs, ns * dofs)).tocsr()
    M.sum_duplicates()
    return M
