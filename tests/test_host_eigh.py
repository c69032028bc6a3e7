"""The library's host Hermitian eigensolvers (used by the Rayleigh-Ritz steps of the
coarsest, fine-level and difference-level eigensolvers), built from their C++ source with
g++ and checked against numpy's LAPACK eigh (CPU).

For random Hermitian matrices (also with clustered and exactly repeated eigenvalues, a
zero matrix, a diagonal one and orders 1 and 2): eigenvalues ascending and within
1e-13 ||A|| of LAPACK's, eigenvectors orthonormal to 1e-13 and A Z = Z diag(w) to 1e-13 ||A||.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2211_15383_amd", "csrc")


@pytest.fixture(scope="module")
def driver():
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "eigh_driver")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "eigh_driver.cpp"),
                    os.path.join(CSRC, "eigh_host.cpp"), "-o", exe], check=True)
    yield exe
    shutil.rmtree(d)


def _run(exe, method, A):
    n = A.shape[0]
    inp = np.int32(n).tobytes() + np.ascontiguousarray(A, dtype=np.complex128).tobytes()
    out = subprocess.run([exe, method], input=inp, capture_output=True, check=True).stdout
    w = np.frombuffer(out[: 8 * n], dtype=np.float64)
    Z = np.frombuffer(out[8 * n:], dtype=np.complex128).reshape(n, n)
    return w, Z


def _hermitian(n, seed, spectrum=None):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    if spectrum is None:
        return (M + M.conj().T) / 2
    Q, _ = np.linalg.qr(M)
    return (Q * spectrum) @ Q.conj().T


CASES = [
    ("order1", lambda: np.array([[2.5 + 0j]])),
    ("order2", lambda: _hermitian(2, 1)),
    ("random50", lambda: _hermitian(50, 2)),
    ("random300", lambda: _hermitian(300, 3)),
    ("clustered", lambda: _hermitian(120, 4, np.concatenate([np.full(40, 1.0), 1.0 + 1e-9 * np.arange(40),
                                                             np.linspace(-3, 3, 40)]))),
    ("repeated", lambda: _hermitian(64, 5, np.repeat([-2.0, 0.5, 7.0, 7.0], 16))),
    ("indefinite_small", lambda: _hermitian(80, 6, np.geomspace(1e-12, 1.0, 80) * np.resize([1, -1], 80))),
    ("zero", lambda: np.zeros((10, 10), dtype=np.complex128)),
    ("diagonal", lambda: np.diag(np.array([3.0, -1.0, 2.0, 0.0, 5.0])).astype(np.complex128)),
]


@pytest.mark.parametrize("method", ["tridiag", "jacobi"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_host_eigh(driver, method, name, make):
    A = make()
    n = A.shape[0]
    if method == "jacobi" and n > 120:
        pytest.skip("Jacobi is the small-order solver")
    w, Z = _run(driver, method, A)
    ref = np.linalg.eigvalsh(A)
    scale = max(np.linalg.norm(A, 2), 1e-300)
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - ref).max() <= 1e-13 * scale
    assert np.abs(Z.conj().T @ Z - np.eye(n)).max() <= 1e-13 * max(n, 10) ** 0.5
    assert np.abs(A @ Z - Z * w).max() <= 1e-13 * scale * max(n, 10) ** 0.5
