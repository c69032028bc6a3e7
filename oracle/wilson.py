"""The 2D Wilson-Schwinger operator, Gamma5 and free-field closed forms (oracle; test only).

The paper names the operator (Sec. 1, Sec. 4.3: the (1+1)-dimensional Schwinger model,
bare mass m0) and uses its Gamma5-hermiticity (Sec. 2, eq. 7) but does not write it out.
Reading used here, with Wilson parameter r = 1 and two spin components:

    (D psi)(x) = (m0 + 2) psi(x)
                 - 1/2 sum_{mu in {x,t}} [ (1 - s_mu) U_mu(x) psi(x + mu)
                                          + (1 + s_mu) conj(U_mu(x - mu)) psi(x - mu) ]

s_x = sigma_1 = [[0, 1], [1, 0]], s_t = sigma_2 = [[0, -i], [i, 0]],
Gamma5 = sigma_3 = diag(1, -1) (spin 0 has chirality +).  Periodic in x; every t-hop
across the t = Lt-1 <-> 0 boundary picks up a factor -1 (antiperiodic in t).

Canonical index: j = 2 * (x + Lx * t) + spin.  Link angles theta[mu, t, x],
U_mu(x, t) = exp(i theta[mu, t, x]).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SIGMA = {
    0: np.array([[0, 1], [1, 0]], dtype=np.complex128),
    1: np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
}
GAMMA5_SPIN = np.diag([1.0, -1.0]).astype(np.complex128)


def dirac_operator(theta: np.ndarray, m0: float, antiperiodic_t: bool = True) -> sp.csr_matrix:
    """Sparse Wilson-Schwinger D (n x n, n = 2 Lx Lt), assembled hop by hop for all sites."""
    _, Lt, Lx = theta.shape
    n = 2 * Lx * Lt
    t, x = np.meshgrid(np.arange(Lt), np.arange(Lx), indexing="ij")
    here = (x + Lx * t).ravel()
    rows, cols, vals = [], [], []

    def put(block, r_site, c_site, coeff):
        # block: 2x2 spin matrix; coeff: per-site complex factor
        for a in range(2):
            for b in range(2):
                if block[a, b] != 0:
                    rows.append(2 * r_site + a)
                    cols.append(2 * c_site + b)
                    vals.append(block[a, b] * coeff)

    eye = np.eye(2, dtype=np.complex128)
    put(eye, here, here, np.full(here.size, m0 + 2.0, dtype=np.complex128))
    for mu in (0, 1):
        if mu == 0:
            xf, tf, xb, tb = (x + 1) % Lx, t, (x - 1) % Lx, t
        else:
            xf, tf, xb, tb = x, (t + 1) % Lt, x, (t - 1) % Lt
        sign_f = np.ones_like(theta[0])
        sign_b = np.ones_like(theta[0])
        if mu == 1 and antiperiodic_t:
            sign_f[t == Lt - 1] = -1.0      # hop t = Lt-1 -> 0
            sign_b[t == 0] = -1.0           # hop t = 0 -> Lt-1
        U_here = np.exp(1j * theta[mu])                 # U_mu(x)
        U_back = np.exp(-1j * theta[mu][tb, xb])        # conj(U_mu(x - mu))
        put(eye - SIGMA[mu], here, (xf + Lx * tf).ravel(), (-0.5 * sign_f * U_here).ravel())
        put(eye + SIGMA[mu], here, (xb + Lx * tb).ravel(), (-0.5 * sign_b * U_back).ravel())
    D = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    D.sum_duplicates()
    return D


def site(x: int, t: int, Lx: int) -> int:
    return x + Lx * t


def gamma5(n_sites: int, dofs: int) -> sp.csr_matrix:
    """Gamma5 at a level with `dofs` dofs per site: +1 on the first half, -1 on the second.

    At the fine level (dofs = 2) this is sigma_3 on spin; at a coarse level the first N
    dofs of a site come from chirality + and the last N from chirality - (eq. 14).
    """
    half = dofs // 2
    d = np.tile(np.concatenate([np.ones(half), -np.ones(half)]), n_sites)
    return sp.diags(d.astype(np.complex128)).tocsr()


def free_field_momenta(Lx: int, Lt: int, antiperiodic_t: bool = True):
    kx = 2.0 * np.pi * np.arange(Lx) / Lx
    shift = 0.5 if antiperiodic_t else 0.0
    kt = 2.0 * np.pi * (np.arange(Lt) + shift) / Lt
    PX, PT = np.meshgrid(kx, kt, indexing="xy")
    return PX.ravel(), PT.ravel()


def free_field_eigenvalues(Lx: int, Lt: int, m0: float, antiperiodic_t: bool = True) -> np.ndarray:
    """Eigenvalues of D at U = 1 by Fourier transform: a(p) +- i b(p) with
    a = m0 + sum_mu (1 - cos p_mu), b = sqrt(sum_mu sin^2 p_mu)."""
    px, pt = free_field_momenta(Lx, Lt, antiperiodic_t)
    a = m0 + (1 - np.cos(px)) + (1 - np.cos(pt))
    b = np.sqrt(np.sin(px) ** 2 + np.sin(pt) ** 2)
    return np.concatenate([a + 1j * b, a - 1j * b])


def free_field_trace_inverse(Lx: int, Lt: int, m0: float, antiperiodic_t: bool = True) -> float:
    """tr(D^-1) at U = 1: sum_p 2 a / (a^2 + b^2)."""
    px, pt = free_field_momenta(Lx, Lt, antiperiodic_t)
    a = m0 + (1 - np.cos(px)) + (1 - np.cos(pt))
    b2 = np.sin(px) ** 2 + np.sin(pt) ** 2
    return float(np.sum(2.0 * a / (a * a + b2)))


def free_field_singular_values(Lx: int, Lt: int, m0: float, antiperiodic_t: bool = True) -> np.ndarray:
    """Singular values of D at U = 1: sqrt(a^2 + b^2), each twice (D(p) is normal)."""
    ev = free_field_eigenvalues(Lx, Lt, m0, antiperiodic_t)
    return np.sort(np.abs(ev))


def gauge_transform(theta: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """Link angles after the gauge transformation g(x) = exp(i alpha(x)):
    U'_mu(x) = g(x) U_mu(x) conj(g(x + mu)), so that D' = G D G^H (G = diag(g) on spin)."""
    _, Lt, Lx = theta.shape
    out = theta.copy()
    out[0] += alpha - np.roll(alpha, -1, axis=1)
    out[1] += alpha - np.roll(alpha, -1, axis=0)
    return out
