"""FP64 NumPy oracle of the silhouette blend and the IoU silhouette loss.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Silhouette blending (paper, Section 3.2, Algorithm 1): per pixel,
prob_k = sigmoid(-dists_k / sigma) and alpha = 1 - prod_k (1 - prob_k).
Reading: slots with no face (p2f == -1) contribute prob_k = 0; otherwise the
-1 padding of dists would make every empty pixel opaque.

IoU loss (paper, Appendix B, "Losses"): per view,
IoU = sum_p S*T / sum_p (S + T - S*T) and the loss is 1 - IoU; the batch loss
is the mean over views.
"""
from __future__ import annotations

import numpy as np


def _sigmoid(x):
    # numerically safe logistic in float64
    out = np.empty_like(x)
    pos = x >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-x[pos]))
    ex = np.exp(x[~pos])
    out[~pos] = ex / (1.0 + ex)
    return out


def silhouette_blend(p2f, dists, sigma):
    """alpha (N,H,W) float64 from p2f (N,H,W,K) and dists (N,H,W,K)."""
    d = np.asarray(dists, dtype=np.float64)
    valid = np.asarray(p2f) >= 0
    prob = np.where(valid, _sigmoid(-d / sigma), 0.0)
    return 1.0 - np.prod(1.0 - prob, axis=-1)


def silhouette_blend_backward(p2f, dists, sigma, grad_alpha):
    """d(sum grad_alpha * alpha)/d dists, float64 (N,H,W,K).

    d alpha / d dists_k = -(1/sigma) prob_k (1 - prob_k) prod_{j != k} (1 - prob_j),
    with the product over j != k formed directly (no division), and zero for
    empty slots.  1 - prob_k is evaluated as sigmoid(+dists_k / sigma).
    """
    d = np.asarray(dists, dtype=np.float64)
    valid = np.asarray(p2f) >= 0
    prob = np.where(valid, _sigmoid(-d / sigma), 0.0)
    one_minus = np.where(valid, _sigmoid(d / sigma), 1.0)
    K = d.shape[-1]
    out = np.zeros_like(d)
    for k in range(K):
        others = np.delete(one_minus, k, axis=-1)
        excl = np.prod(others, axis=-1)
        out[..., k] = -(1.0 / sigma) * prob[..., k] * one_minus[..., k] * excl
    out = np.where(valid, out, 0.0)
    return out * np.asarray(grad_alpha, dtype=np.float64)[..., None]


def iou_loss(alpha, target):
    """mean over views of 1 - sum(S*T) / sum(S + T - S*T); alpha/target (N,H,W)."""
    S = np.asarray(alpha, dtype=np.float64)
    T = np.asarray(target, dtype=np.float64)
    inter = (S * T).reshape(S.shape[0], -1).sum(1)
    union = (S + T - S * T).reshape(S.shape[0], -1).sum(1)
    return float(np.mean(1.0 - inter / union))
