"""Pins of the checker's Wilson-Schwinger operator (CPU).

* Gamma5-hermiticity Gamma5 D Gamma5 = D^H (Sec. 2, the relation used for eq. 7).
* Free field (U = 1): eigenvalues a(p) +- i b(p) and tr(D^-1) in closed form by Fourier
  transform, with antiperiodic momenta in t; catches wrong spin matrices, hop signs,
  boundary phases and mass convention.
* Gauge covariance D[g.U] = G D G^H: catches a link taken at the wrong site on either hop.
* sigma_min(D) = min |lambda(Gamma5 D)| (eq. 7).
"""
import numpy as np
import pytest

from oracle import wilson
from paper_2211_15383_amd.inputs import link_angles


def _sorted(v):
    return v[np.lexsort((np.round(v.imag, 9), np.round(v.real, 9)))]


@pytest.mark.parametrize("Lx,Lt,seed", [(4, 4, 1), (6, 4, 2), (3, 5, 3), (8, 8, 4)])
def test_gamma5_hermiticity(Lx, Lt, seed):
    D = wilson.dirac_operator(link_angles(Lx, Lt, 0.7, seed), -0.3)
    G = wilson.gamma5(Lx * Lt, 2)
    assert abs(G @ D @ G - D.conj().T).max() == 0.0


@pytest.mark.parametrize("Lx,Lt,m0,ap", [(6, 4, 0.05, True), (8, 8, -0.2, True), (5, 6, 0.3, False)])
def test_free_field_spectrum(Lx, Lt, m0, ap):
    D = wilson.dirac_operator(np.zeros((2, Lt, Lx)), m0, antiperiodic_t=ap).toarray()
    ev = np.linalg.eigvals(D)
    cf = wilson.free_field_eigenvalues(Lx, Lt, m0, antiperiodic_t=ap)
    assert np.abs(_sorted(ev) - _sorted(cf)).max() < 1e-13


@pytest.mark.parametrize("Lx,Lt,m0", [(8, 8, 0.1), (12, 6, -0.05)])
def test_free_field_trace(Lx, Lt, m0):
    D = wilson.dirac_operator(np.zeros((2, Lt, Lx)), m0).toarray()
    tr = np.trace(np.linalg.inv(D))
    cf = wilson.free_field_trace_inverse(Lx, Lt, m0)
    assert abs(tr.imag) < 1e-12 * abs(cf)
    assert abs(tr.real - cf) < 1e-12 * abs(cf)


def test_free_field_singular_values():
    D = wilson.dirac_operator(np.zeros((2, 8, 6)), 0.02).toarray()
    sv = np.sort(np.linalg.svd(D, compute_uv=False))
    assert np.abs(sv - wilson.free_field_singular_values(6, 8, 0.02)).max() < 1e-13


def test_gauge_covariance():
    theta = link_angles(6, 8, 0.5, 9)
    alpha = np.random.default_rng(5).uniform(-np.pi, np.pi, size=(8, 6))
    D = wilson.dirac_operator(theta, -0.1).toarray()
    Dg = wilson.dirac_operator(wilson.gauge_transform(theta, alpha), -0.1).toarray()
    g = np.repeat(np.exp(1j * alpha.ravel()), 2)
    assert np.abs(g[:, None] * D * g.conj()[None, :] - Dg).max() < 1e-14
    assert abs(np.trace(np.linalg.inv(D)) - np.trace(np.linalg.inv(Dg))) < 1e-11


def test_sigma_min_from_gamma5_eigenvalues():
    theta = link_angles(8, 8, 0.3, 1)
    D = wilson.dirac_operator(theta, -0.08)
    sv = np.linalg.svd(D.toarray(), compute_uv=False)
    ev = np.linalg.eigvalsh((wilson.gamma5(64, 2) @ D).toarray())
    assert np.abs(np.sort(sv) - np.sort(np.abs(ev))).max() < 1e-13


def test_stencil_structure():
    """Nine entries per row; the diagonal is m0 + 2."""
    D = wilson.dirac_operator(link_angles(6, 6, 0.3, 2), 0.25)
    assert np.all(np.diff(D.indptr) == 9)
    assert np.allclose(D.diagonal(), 2.25, rtol=0, atol=0)
