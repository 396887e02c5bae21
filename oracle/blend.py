"""FP64 NumPy oracle of the silhouette blend and the IoU silhouette loss.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Silhouette blending (paper, Section 3.2, Algorithm 1): per pixel,
prob_k = sigmoid(-dists_k / sigma) and alpha = 1 - prod_k (1 - prob_k).
Reading: slots with no face (p2f == -1) contribute prob_k = 0; otherwise the
-1 padding of dists would make every empty pixel opaque.

Softmax blending (paper, Section 3.2, Algorithm 2): per pixel,
prob_k = sigmoid(-dists_k / sigma), zinv_k = (zfar - zbuf_k) / (zfar - znear),
weights_k = prob_k exp((zinv_k - max_j zinv_j) / gamma), normalised to sum 1,
image = sum_k weights_k colors_k.  Readings: slots with no face take no part
(no weight and no say in the maximum); a pixel whose weights sum to 0 (no
face, or every prob underflowing) is 0.

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


def _softmax_parts(p2f, zbuf, dists, sigma, gamma, znear, zfar):
    valid = np.asarray(p2f) >= 0
    d = np.asarray(dists, np.float64)
    z = np.asarray(zbuf, np.float64)
    prob = np.where(valid, _sigmoid(-d / sigma), 0.0)
    zinv = (zfar - z) / (zfar - znear)
    zmax = np.max(np.where(valid, zinv, -np.inf), axis=-1, keepdims=True)
    zmax = np.where(np.isfinite(zmax), zmax, 0.0)
    w = np.where(valid, prob * np.exp(np.where(valid, zinv - zmax, 0.0) / gamma), 0.0)
    return valid, prob, w, w.sum(-1)


def softmax_blend(p2f, zbuf, dists, colors, sigma, gamma, znear, zfar):
    """image (N,H,W,C) float64 from Fragments (N,H,W,K) and colors (N,H,W,K,C)."""
    _, _, w, W = _softmax_parts(p2f, zbuf, dists, sigma, gamma, znear, zfar)
    c = np.asarray(colors, np.float64)
    num = (w[..., None] * c).sum(-2)
    safe = np.where(W > 0, W, 1.0)
    return np.where((W > 0)[..., None], num / safe[..., None], 0.0)


def softmax_blend_backward(p2f, zbuf, dists, colors, sigma, gamma, znear, zfar, grad_image):
    """(grad_zbuf, grad_dists, grad_colors) of sum(grad_image * image), float64.

    With W = sum_k w_k and image_c = sum_k w_k colors_kc / W:
      G_k = sum_c grad_c (colors_kc - image_c) / W      (d L / d w_k)
      d L / d dists_k = -G_k w_k (1 - prob_k) / sigma
      d L / d zbuf_k  = -G_k w_k / (gamma (zfar - znear))
      d L / d colors_kc = grad_c w_k / W
    The shift by max zinv cancels in the normalised weights, so it carries no
    gradient.  Empty slots and pixels with W = 0 get zero gradients.
    """
    valid, prob, w, W = _softmax_parts(p2f, zbuf, dists, sigma, gamma, znear, zfar)
    c = np.asarray(colors, np.float64)
    g = np.asarray(grad_image, np.float64)
    img = softmax_blend(p2f, zbuf, dists, colors, sigma, gamma, znear, zfar)
    safe = np.where(W > 0, W, 1.0)
    live = (W > 0)
    G = np.where(live[..., None], ((c - img[..., None, :]) * g[..., None, :]).sum(-1) / safe[..., None], 0.0)
    one_minus = _sigmoid(np.asarray(dists, np.float64) / sigma)  # 1 - prob, accurate where prob ~ 1
    gd = np.where(valid, -G * w * one_minus / sigma, 0.0)
    gz = np.where(valid, -G * w / (gamma * (zfar - znear)), 0.0)
    gc = np.where((valid & live[..., None])[..., None], g[..., None, :] * (w / safe[..., None])[..., None], 0.0)
    return gz, gd, gc
