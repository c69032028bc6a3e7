"""Shared helpers of the GPU tests: oracle hierarchies, GPU hierarchies built from the
same test vectors, tensor conversions, error measures."""
import functools

import numpy as np

from oracle import deflation as odfl, multigrid as omg
from paper_2211_15383_amd.inputs import WORKLOADS, load_m0


@functools.lru_cache(maxsize=None)
def oracle_hierarchy(name: str):
    W = WORKLOADS[name]
    m0 = load_m0(name)
    lv = omg.build_hierarchy(W.theta(), m0, W.aggs, W.ntv, W.n_inv, W.mg_seed)
    return W, m0, lv


@functools.lru_cache(maxsize=None)
def oracle_deflation(name: str, k: int):
    W, m0, lv = oracle_hierarchy(name)
    return odfl.deflate(lv[-1].D, lv[-1].gamma5, k)


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def to_dev(torch, x: np.ndarray, dtype=None):
    """numpy [n, nrhs] (columns = vectors) -> torch [nrhs, n] on cuda:0."""
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(x).T))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def to_host(t) -> np.ndarray:
    """torch [nrhs, n] -> numpy [n, nrhs] complex128."""
    return t.detach().cpu().numpy().astype(np.complex128).T


def random_vectors(n: int, m: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, m)) + 1j * rng.normal(size=(n, m))
