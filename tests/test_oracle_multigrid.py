"""Pins of the checker's multigrid hierarchy (CPU).

* P^H P = I (stated before eq. 11) and P P^H V = V: each test vector lies in the range of
  its aggregate-chirality block (the local QR keeps the span).
* Spin-preserving relations Gamma5^l P_l = P_l Gamma5^{l+1} and the Hermitian Q_l
  (eq. 14); coarse Gamma5-hermiticity follows.
* The explicit product P^H D P is a nearest-neighbour block stencil (five blocks per
  site) and the block representation reproduces it exactly.
* The global MGS between inverse-iteration steps does not change P (it only right-
  multiplies by an upper-triangular matrix with positive diagonal).
* Free field with constant test vectors: P^H D P is the Fourier-diagonal free operator
  of the coarse lattice's constant mode (a closed form for one coarse block).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import multigrid as mg, wilson
from paper_2211_15383_amd.inputs import WORKLOADS, link_angles


def _hier(name, m0=-0.05):
    W = WORKLOADS[name]
    return W, mg.build_hierarchy(W.theta(), m0, W.aggs, W.ntv, W.n_inv, W.mg_seed)


@pytest.mark.parametrize("name", ["schwinger16", "tiny8x16", "rect24x16"])
def test_orthonormal_and_spans_test_vectors(name):
    W, lv = _hier(name)
    for l in range(len(lv) - 1):
        P = lv[l].P
        assert abs(P.conj().T @ P - np.eye(P.shape[1])).max() < 1e-14
        V = lv[l].V
        assert np.abs(P @ (P.conj().T @ V) - V).max() < 1e-12 * np.abs(V).max()


@pytest.mark.parametrize("name", ["schwinger16", "tiny8x16", "rect24x16"])
def test_spin_preserving_relations(name):
    W, lv = _hier(name)
    for l in range(len(lv) - 1):
        G, Gc, P = lv[l].gamma5, lv[l + 1].gamma5, lv[l].P
        assert abs(G @ P - P @ Gc).max() == 0.0
        assert abs(P.conj().T @ G - Gc @ P.conj().T).max() == 0.0
    for l in range(len(lv)):
        G, D = lv[l].gamma5, lv[l].D
        Q = G @ D
        assert abs(Q - Q.conj().T).max() < 1e-13


@pytest.mark.parametrize("name", ["schwinger16", "rect24x16"])
def test_coarse_operator_is_block_stencil(name):
    W, lv = _hier(name)
    for l in range(1, len(lv)):
        c = lv[l]
        A = mg.coarse_blocks(c.D, c.Lx, c.Lt, c.dofs)
        assert A.shape == (c.Lx * c.Lt, 5, c.dofs, c.dofs)
        assert abs(mg.blocks_to_sparse(A, c.Lx, c.Lt) - c.D).max() == 0.0


def test_extent_two_lumps_couplings():
    """On a coarse lattice of extent 2 the +mu and -mu neighbours coincide."""
    W, lv = _hier("rect24x16")
    c = lv[2]
    assert (c.Lx, c.Lt) == (2, 2)
    A = mg.coarse_blocks(c.D, c.Lx, c.Lt, c.dofs)
    assert np.all(A[:, 2] == 0) and np.all(A[:, 4] == 0)
    assert np.abs(A[:, 1]).max() > 0 and np.abs(A[:, 3]).max() > 0


def test_mgs_between_steps_does_not_change_P():
    W = WORKLOADS["schwinger16"]
    lv = mg.build_hierarchy(W.theta(), -0.05, W.aggs, W.ntv, 2, W.mg_seed)
    D = lv[0].D
    V0 = mg.start_vectors(W.mg_seed, 1, W.ntv[0], D.shape[0])
    lu = spla.splu(D.tocsc())
    V = lu.solve(lu.solve(V0))                  # D^-2 V0, no orthogonalisation
    P2 = mg.interpolator(V, 16, 16, 2, 4, 4)
    assert abs(P2 - lv[0].P).max() < 1e-9


def test_free_field_constant_vectors():
    """U = 1, test vectors constant per chirality: each coarse self block is
    (m0 + 2) I - (hops inside the aggregate), and coarse hop blocks are the fine hop
    spin matrices scaled by (boundary sites) / (aggregate sites)."""
    Lx = Lt = 8
    a = 2
    m0 = 0.3
    D = wilson.dirac_operator(np.zeros((2, Lt, Lx)), m0, antiperiodic_t=False)
    V = np.zeros((2 * Lx * Lt, 1), dtype=np.complex128)
    V[:, 0] = 1.0
    P = mg.interpolator(V, Lx, Lt, 2, a, a)
    A = mg.coarse_blocks(mg.galerkin(D, P), Lx // a, Lt // a, 2)
    s1, s2 = wilson.SIGMA[0], wilson.SIGMA[1]
    eye = np.eye(2)
    # per direction: a*(a-1) internal hop pairs out of a*a sites; a boundary hops out of a*a
    inner = (a * (a - 1)) / (a * a)
    bnd = a / (a * a)
    self_blk = (m0 + 2) * eye - 0.5 * inner * ((eye - s1) + (eye + s1) + (eye - s2) + (eye + s2))
    for s in range(A.shape[0]):
        assert np.abs(A[s, 0] - self_blk).max() < 1e-14
        assert np.abs(A[s, 1] + 0.5 * bnd * (eye - s1)).max() < 1e-14
        assert np.abs(A[s, 2] + 0.5 * bnd * (eye + s1)).max() < 1e-14
        assert np.abs(A[s, 3] + 0.5 * bnd * (eye - s2)).max() < 1e-14
        assert np.abs(A[s, 4] + 0.5 * bnd * (eye + s2)).max() < 1e-14


def test_geometry_validation():
    with pytest.raises(ValueError):
        mg.check_geometry(10, 8, 2, 4, 4, 2)      # 10 not divisible by 4
    with pytest.raises(ValueError):
        mg.check_geometry(4, 8, 2, 4, 4, 2)       # coarse extent 1
    with pytest.raises(ValueError):
        mg.check_geometry(8, 8, 2, 2, 2, 5)       # 4 rows per block < 5 vectors
