"""FP64 NumPy oracle of the point-cloud compositing (paper, Section 3.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a pixel covered by points with opacities alpha_1..alpha_K in increasing
z and features f_1..f_K (rows of a (P, D) feature table, picked by idx):
  Alpha compositing: f = sum_i alpha_i prod_{j<i} (1 - alpha_j) f_i
  Norm (normalised weighted sum): f = sum_i alpha_i f_i / sum_i alpha_i
Readings: slots with idx == -1 take no part; a pixel whose opacities sum to 0
gets 0 under Norm.
"""
from __future__ import annotations

import numpy as np


def splat_alpha(idx, dists, radius):
    """Opacity of a splat at squared distance d from its point (a reading: the
    paper only says that it falls away from the centre): 1 - d / r^2, from 1
    at the point to 0 at the rim; 0 for empty slots."""
    idx = np.asarray(idx)
    d = np.asarray(dists, np.float64)
    r2 = float(radius) * float(radius)
    return np.where(idx >= 0, 1.0 - d / r2, 0.0)


def _gather(idx, features):
    idx = np.asarray(idx)
    feat = np.asarray(features, np.float64)
    valid = idx >= 0
    g = feat[np.where(valid, idx, 0)]
    return valid, np.where(valid[..., None], g, 0.0)


def alpha_composite(idx, alphas, features):
    """(N,H,W,D) from idx (N,H,W,K), alphas (N,H,W,K), features (P,D)."""
    valid, f = _gather(idx, features)
    a = np.where(valid, np.asarray(alphas, np.float64), 0.0)
    K = a.shape[-1]
    out = np.zeros(a.shape[:-1] + (f.shape[-1],))
    trans = np.ones(a.shape[:-1])
    for k in range(K):
        out += (a[..., k] * trans)[..., None] * f[..., k, :]
        trans = trans * (1.0 - a[..., k])
    return out


def alpha_composite_backward(idx, alphas, features, grad_out):
    """(grad_alphas (N,H,W,K), grad_features (P,D)) of sum(grad_out * f_Alpha).

    With T_k = prod_{j<k} (1 - alpha_j) and g_k = <grad_out, f_k>:
      d/d alpha_k = T_k g_k - sum_{i>k} alpha_i T_i g_i / (1 - alpha_k)
    formed without the division as T_k g_k - sum_{i>k} alpha_i g_i prod_{j<i, j!=k} (1 - alpha_j);
      d/d f_k = alpha_k T_k grad_out (scattered to the feature rows)."""
    valid, f = _gather(idx, features)
    a = np.where(valid, np.asarray(alphas, np.float64), 0.0)
    g = np.asarray(grad_out, np.float64)
    K = a.shape[-1]
    gdot = (f * g[..., None, :]).sum(-1)                 # (N,H,W,K)
    ga = np.zeros_like(a)
    for k in range(K):
        Tk = np.prod(1.0 - a[..., :k], axis=-1)
        acc = Tk * gdot[..., k]
        for i in range(k + 1, K):
            others = np.prod(np.delete(1.0 - a[..., :i], k, axis=-1), axis=-1)
            acc = acc - a[..., i] * gdot[..., i] * others
        ga[..., k] = acc
    ga = np.where(valid, ga, 0.0)
    feat = np.asarray(features, np.float64)
    gf = np.zeros_like(feat)
    idx = np.asarray(idx)
    T = np.ones(a.shape[:-1])
    for k in range(K):
        w = (a[..., k] * T)[..., None] * g                    # (N,H,W,D)
        sel = valid[..., k]
        np.add.at(gf, idx[..., k][sel], w[sel])
        T = T * (1.0 - a[..., k])
    return ga, gf


def norm_composite(idx, alphas, features):
    """(N,H,W,D): sum alpha f / sum alpha over filled slots, 0 where the sum is 0."""
    valid, f = _gather(idx, features)
    a = np.where(valid, np.asarray(alphas, np.float64), 0.0)
    s = a.sum(-1)
    num = (a[..., None] * f).sum(-2)
    return np.where((s > 0)[..., None], num / np.where(s > 0, s, 1.0)[..., None], 0.0)


def norm_composite_backward(idx, alphas, features, grad_out):
    """(grad_alphas, grad_features) of sum(grad_out * f_Norm):
    d/d alpha_k = <grad_out, f_k - f_Norm> / S, d/d f_k = alpha_k grad_out / S."""
    valid, f = _gather(idx, features)
    a = np.where(valid, np.asarray(alphas, np.float64), 0.0)
    g = np.asarray(grad_out, np.float64)
    s = a.sum(-1)
    live = s > 0
    safe = np.where(live, s, 1.0)
    out = norm_composite(idx, alphas, features)
    ga = np.where(valid & live[..., None], ((f - out[..., None, :]) * g[..., None, :]).sum(-1) / safe[..., None], 0.0)
    feat = np.asarray(features, np.float64)
    gf = np.zeros_like(feat)
    idx = np.asarray(idx)
    for k in range(a.shape[-1]):
        sel = valid[..., k] & live
        w = (a[..., k] / safe)[..., None] * g
        np.add.at(gf, idx[..., k][sel], w[sel])
    return ga, gf
