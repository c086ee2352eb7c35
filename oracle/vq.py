"""Vector quantisation of the SH coefficients (the post-processing of Sec. 5,
"Ours-PP": each Gaussian's SH is replaced by a codebook entry), FP64.

TEST INFRASTRUCTURE ONLY: the product library never imports this module.

  A Gaussian's SH is the vector of its 16 x 3 coefficients, ordered basis-major
  (k = 0..15, then channel r, g, b), as stored in the model's [16][3][n] planes.
  Codebook: K such vectors.  Quantisation is Lloyd's k-means:
    assign: a(i) = argmin_j ||x_i - c_j||^2, equal distances to the lower j;
    update: c_j = mean of the x_i with a(i) = j; an empty cluster keeps c_j.
  The initial codebook is the vectors of K Gaussians the caller picks.
  Rendering a quantised model is rendering the model whose SH planes hold
  c_{a(i)} for Gaussian i.
"""
from __future__ import annotations

import numpy as np


def sh_vectors(sh_planes) -> np.ndarray:
    """[16][3][n] planes -> (n, 48) vectors (basis-major, then channel)."""
    sh = np.asarray(sh_planes, dtype=np.float64)
    return np.transpose(sh, (2, 0, 1)).reshape(sh.shape[2], -1)


def planes_from_vectors(vec: np.ndarray) -> np.ndarray:
    """(n, 48) -> [16][3][n]."""
    vec = np.asarray(vec)
    return np.transpose(vec.reshape(vec.shape[0], 16, 3), (1, 2, 0))


def squared_distances(x: np.ndarray, c: np.ndarray) -> np.ndarray:
    """(n, K) matrix of ||x_i - c_j||^2, each the sum of squared differences."""
    d = x[:, None, :] - c[None, :, :]
    return np.einsum("nkd,nkd->nk", d, d)


def assign(x: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Index of the nearest codebook vector (first of equal distances)."""
    out = np.empty(x.shape[0], dtype=np.int64)
    for s in range(0, x.shape[0], 4096):
        out[s:s + 4096] = np.argmin(squared_distances(x[s:s + 4096], c), axis=1)
    return out


def update(x: np.ndarray, a: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Cluster means; an empty cluster keeps its vector."""
    k = c.shape[0]
    sums = np.zeros_like(c, dtype=np.float64)
    np.add.at(sums, a, x)
    counts = np.bincount(a, minlength=k)
    out = np.array(c, dtype=np.float64)
    nz = counts > 0
    out[nz] = sums[nz] / counts[nz, None]
    return out


def kmeans(x: np.ndarray, init_index, iterations: int):
    """Lloyd iterations from the vectors at init_index; returns (codebook,
    assignment of the last codebook)."""
    x = np.asarray(x, dtype=np.float64)
    c = x[np.asarray(init_index, dtype=np.int64)].copy()
    for _ in range(iterations):
        c = update(x, assign(x, c), c)
    return c, assign(x, c)


def inertia(x: np.ndarray, c: np.ndarray, a: np.ndarray) -> float:
    """Sum of squared distances to the assigned vectors."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(c, dtype=np.float64)[a]
    return float(np.sum(d * d))
