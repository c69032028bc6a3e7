"""Bare-mass rule of the synthetic workloads: m0 such that sigma_min(D) ~ 1e-2 (oracle; test only).

The paper runs near-critical (m0 = -0.1320 on its own 128^2 configuration, Sec. 4.3),
where the smallest singular values dominate the Hutchinson variance (Sec. 2, eq. 3).  On
the synthetic i.i.d. links the same regime is set by a rule:

* sigma_min(m) = min |lambda(Gamma5 D(m))| (Gamma5-hermiticity, eq. 7);
* scan down from m_start (default +0.1) in steps of 0.005 to the first m with
  sigma_min < 1e-2 (sigma_min is not monotone through the critical mass, so the small
  step keeps the first crossing), then shrink the bracket between the last two scan
  points by the Illinois variant of regula falsi on sigma_min(m) - 1e-2, keeping the
  endpoint with sigma_min >= 1e-2, until |sigma_min / 1e-2 - 1| < 1e-3 (at most 40
  steps); that endpoint is m0;
* on lattices too small to reach 1e-2 (the antiperiodic finite-volume gap keeps
  sigma_min above ~2/L for smooth fields) the scan instead stops once sigma_min has risen
  on two consecutive steps, and m0 is the minimiser of sigma_min, refined by
  golden-section search to 1e-5 in m (the most ill-conditioned mass).

sigma_min is computed by dense eigvalsh for n <= 4096, else by shift-invert Lanczos
(scipy eigsh, sigma = 0) on Gamma5 D, whose sparse LU is taken in a geometric nested-
dissection order of the sites (a permutation only: it changes the fill, not the result).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import wilson

TARGET = 1e-2


def nested_dissection_sites(Lx: int, Lt: int) -> np.ndarray:
    """Site elimination order for the torus: separator columns x = 0, Lx/2 and rows
    t = 0, Lt/2 last, the four open rectangles recursively bisected in between."""
    order = []

    def rect(x0, x1, t0, t1):
        w, h = x1 - x0, t1 - t0
        if w <= 0 or h <= 0:
            return
        if w * h <= 16:
            order.extend(x + Lx * t for t in range(t0, t1) for x in range(x0, x1))
        elif w >= h:
            xm = x0 + w // 2
            rect(x0, xm, t0, t1)
            rect(xm + 1, x1, t0, t1)
            order.extend(xm + Lx * t for t in range(t0, t1))
        else:
            tm = t0 + h // 2
            rect(x0, x1, t0, tm)
            rect(x0, x1, tm + 1, t1)
            order.extend(x + Lx * tm for x in range(x0, x1))

    hx, ht = Lx // 2, Lt // 2
    seps = []
    for a, b in ((1, hx), (hx + 1, Lx)):
        rect(a, b, 1, ht)
        rect(a, b, ht + 1, Lt)
        seps.extend(x + Lx * t for t in (0, ht) for x in range(a, b))
    seps.extend(x + Lx * t for x in (0, hx) for t in range(Lt))
    order.extend(seps)
    out = np.array(order, dtype=np.int64)
    if out.size != Lx * Lt or np.unique(out).size != Lx * Lt:
        raise AssertionError("nested dissection order is not a permutation")
    return out


def sigma_min(theta: np.ndarray, m: float, method: str = "auto") -> float:
    _, Lt, Lx = theta.shape
    D = wilson.dirac_operator(theta, m)
    Q = wilson.gamma5(Lx * Lt, 2) @ D
    if method == "dense" or (method == "auto" and Q.shape[0] <= 4096):
        return float(np.min(np.abs(np.linalg.eigvalsh(Q.toarray()))))
    s = nested_dissection_sites(Lx, Lt)
    p = np.stack([2 * s, 2 * s + 1], axis=1).ravel()
    Qp = Q.tocsr()[p][:, p].tocsc()
    lu = spla.splu(Qp, permc_spec="NATURAL", diag_pivot_thresh=0.0)
    op = spla.LinearOperator(Qp.shape, matvec=lu.solve, dtype=np.complex128)
    vals = spla.eigsh(Qp, k=1, sigma=0.0, which="LM", OPinv=op, return_eigenvectors=False)
    return float(np.min(np.abs(vals)))


def scan_points(m_start: float, step: float, count: int):
    """The first `count` masses the scan of m0_rule visits, computed as it computes them."""
    out, m = [m_start], m_start
    for _ in range(count - 1):
        m = m - step
        out.append(m)
    return out


def m0_rule(theta: np.ndarray, m_start: float = 0.1, step: float = 0.005, target: float = TARGET,
            sigma_fn=None):
    """Returns (m0, sigma_min(m0), kind) with kind "crossing" or "minimum".

    sigma_fn: optional callable m -> sigma_min(theta, m) used instead of computing each
    value here (for instance a table filled in parallel, or a recorded one)."""
    def smin(m):
        return sigma_min(theta, m) if sigma_fn is None else sigma_fn(m)

    m_prev, s_prev = m_start, smin(m_start)
    if s_prev < target:
        raise ValueError("sigma_min already below target at the scan start")
    history = [(m_prev, s_prev)]
    rises = 0
    while True:
        m_cur = m_prev - step
        s_cur = smin(m_cur)
        history.append((m_cur, s_cur))
        if s_cur < target:
            m_hi, s_hi, m_lo, s_lo = m_prev, s_prev, m_cur, s_cur
            side = 0
            for _ in range(40):
                if abs(s_hi / target - 1.0) < 1e-3:
                    break
                f_hi, f_lo = s_hi - target, s_lo - target
                if side == 1:
                    f_lo *= 0.5
                elif side == -1:
                    f_hi *= 0.5
                m_new = m_hi - f_hi * (m_hi - m_lo) / (f_hi - f_lo)
                s_new = smin(m_new)
                if s_new >= target:
                    m_hi, s_hi = m_new, s_new
                    side = 1
                else:
                    m_lo, s_lo = m_new, s_new
                    side = -1
            return m_hi, s_hi, "crossing"
        rises = rises + 1 if s_cur > s_prev else 0
        if rises >= 2:
            break
        m_prev, s_prev = m_cur, s_cur
        if m_cur < m_start - 2.0:
            raise ValueError("no crossing and no minimum found")
    # bracket the minimiser: the scan point with the smallest sigma_min and its neighbours
    i = min(range(len(history)), key=lambda j: history[j][1])
    a, b = history[i][0] + step, history[i][0] - step
    g = (np.sqrt(5.0) - 1.0) / 2.0
    c, d = b + g * (a - b), a - g * (a - b)
    fc, fd = smin(c), smin(d)
    while abs(a - b) > 1e-5:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b + g * (a - b)
            fc = smin(c)
        else:
            a, c, fc = c, d, fd
            d = a - g * (a - b)
            fd = smin(d)
    m = 0.5 * (a + b)
    return m, smin(m), "minimum"
