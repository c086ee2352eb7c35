"""Spatial-temporal variation score and pruning (Sec. 4.2.1, Eq. 4-7), FP64.

TEST INFRASTRUCTURE ONLY: the product library never imports this module.

  Spatial score (Eq. 4): S^S_i = sum over every pixel of every scored view of
      alpha_i T_i, the weight Gaussian i receives in that pixel's blend
      (Eq. 2); views are (camera, time) pairs and the sum runs over all of them.
  Temporal score (Eq. 5-6): p_i''(t) = ((t - mu_t)^2 / Sigma_t^2 - 1 / Sigma_t) p_i(t)
      with Sigma_t = Sigma_44 (a variance) and p_i(t) of Eq. 3;
      S^TV_i = sum over the scored times t of 1 / (0.5 tanh(|p_i''(t)|) + 0.5).
  Volume weight (the normalisation the paper borrows): V_i = prod_k s_k, the
      4D volume up to a constant; gamma_i = min(V_i / V_90, 1)^beta with V_90
      the volume at the 90 % position of the ascending volumes
      (index floor(0.9 (n - 1))) and beta = 0.1.
  Score (Eq. 7): S_i = S^TV_i gamma_i S^S_i (S^T_i = S^TV_i gamma_i does not
      depend on t, so the sum over t of Eq. 7 is carried by S^S).
  Pruning: keep the n_keep highest scores, equal scores by the lower index;
      the kept indices are returned in ascending order.
"""
from __future__ import annotations

import math

import numpy as np

from .composite import Settings, composite, prepare
from .slicing import covariance_4d, rows, valid_gaussians


def spatial_score(scene_arrays, views, st: Settings, with_slack: bool = False):
    """views: sequence of (camera, t).  Returns S^S (float64[n]); with_slack=True
    returns (S^S, slack), slack being the most a float32 renderer's score may
    differ because of the pixels whose decisions sit near a threshold."""
    n = scene_arrays[0].shape[1]
    score = np.zeros(n)
    slack = np.zeros(n)
    for cam, t in views:
        pre = prepare(scene_arrays, cam, float(t), st)
        img = composite(pre, cam, st, mode="rect", weights=True)
        score += img.weight
        slack += img.weight_slack
    return (score, slack) if with_slack else score


def temporal_second_derivative(t, mu_t, sigma44):
    """Eq. 5."""
    d = np.asarray(t, dtype=np.float64) - mu_t
    p = np.exp(-d * d / (2.0 * sigma44))
    return (d * d / (sigma44 * sigma44) - 1.0 / sigma44) * p


def temporal_variation_score(mu_t, sigma44, times) -> np.ndarray:
    """Eq. 6."""
    acc = np.zeros(np.shape(mu_t))
    for t in times:
        acc += 1.0 / (0.5 * np.tanh(np.abs(temporal_second_derivative(float(t), mu_t, sigma44))) + 0.5)
    return acc


def volume_weight(log_scale_rows: np.ndarray, valid: np.ndarray, beta: float = 0.1,
                  quantile: float = 0.9) -> np.ndarray:
    """gamma_i = min(V_i / V_q, 1)^beta, V_i = exp(sum of the four log scales);
    invalid Gaussians get V = 0."""
    vol = np.where(valid, np.exp(np.where(valid[:, None], log_scale_rows, 0.0).sum(axis=1)), 0.0)
    n = vol.shape[0]
    if n == 0:
        return vol
    vq = np.sort(vol)[int(math.floor(quantile * (n - 1)))]
    if not vq > 0.0:
        return np.where(vol > 0.0, 1.0, 0.0)
    return np.minimum(vol / vq, 1.0) ** beta


def variation_score(scene_arrays, spatial: np.ndarray, times) -> np.ndarray:
    """Eq. 7: S^TV gamma S^S for every Gaussian (0 for invalid ones)."""
    mean, log_scale, q_l, q_r, logit = scene_arrays[:5]
    M, LS, QL, QR = rows(mean), rows(log_scale), rows(q_l), rows(q_r)
    valid = valid_gaussians(M, LS, QL, QR, np.asarray(logit, dtype=np.float64))
    LS_ = np.where(valid[:, None], LS, 0.0)
    QL_, QR_ = np.where(valid[:, None], QL, 1.0), np.where(valid[:, None], QR, 1.0)
    s44 = covariance_4d(LS_, QL_, QR_)[:, 3, 3]
    tv = temporal_variation_score(np.where(valid, M[:, 3], 0.0), s44, times)
    gamma = volume_weight(LS, valid)
    return np.where(valid, tv * gamma * spatial, 0.0)


def prune(score: np.ndarray, n_keep: int) -> np.ndarray:
    """Ascending indices of the n_keep highest scores (ties: lower index first)."""
    n = score.shape[0]
    n_keep = max(0, min(int(n_keep), n))
    order = np.lexsort((np.arange(n), -np.asarray(score, dtype=np.float64)))
    return np.sort(order[:n_keep]).astype(np.uint32)
