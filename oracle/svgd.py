"""FP64 oracle of the Stein variational gradient descent baseline -- TEST INFRASTRUCTURE
(the import rule of this package applies).

The paper compares its sampler against SVGD (Liu and Wang 2016, cited in the
introduction; the head-to-head comparison of the contributions list and Sec. 3's 2D
experiments: 20 particles, conventional full-shot FWI gradients, null prior, box bounds).
The paper restates no formula; this follows the cited method:
  * particles x_1..x_n (rows), target density p ~ exp(-Phi): grad log p = -grad Phi = -g;
  * RBF kernel k(x, y) = exp(-|x - y|^2 / h);
  * bandwidth by the median heuristic h = med^2 / log n, med^2 read as the median of the
    squared pairwise distances over the pairs i < j (mean of the two middle values when
    their number is even); h = 1 when it is undefined (one particle, or coincident
    particles: median 0);
  * direction phi(x_i) = (1/n) sum_j [k(x_j, x_i) (-g_j) + grad_{x_j} k(x_j, x_i)], where
    grad_{x_j} k(x_j, x_i) = (2/h) (x_i - x_j) k(x_j, x_i) (the repulsive term);
  * step x_i <- clamp(x_i + eps phi(x_i), lo, hi).
"""
from __future__ import annotations

import numpy as np


def sq_distances(x):
    """D[i, j] = sum over cells of (x_i - x_j)^2, written out pair by pair."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            d = x[i] - x[j]
            D[i, j] = D[j, i] = float(np.dot(d, d))
    return D


def bandwidth(D):
    """Median heuristic: median of D over i < j, divided by log n; 1 when that is not a
    positive number (n = 1, or coincident particles)."""
    n = D.shape[0]
    if n < 2:
        return 1.0
    iu = np.triu_indices(n, 1)
    h = float(np.median(D[iu])) / np.log(n)
    return h if 0.0 < h < np.inf else 1.0


def direction(x, g, h=None):
    """(phi [n, N], K [n, n], h) for particles x and misfit gradients g ([n, N] each); h
    None or <= 0 selects the median heuristic."""
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = x.shape[0]
    D = sq_distances(x)
    if h is None or h <= 0:
        h = bandwidth(D)
    K = np.exp(-D / h)
    phi = np.zeros_like(x)
    for i in range(n):
        for j in range(n):
            phi[i] += K[j, i] * (-g[j]) + (2.0 / h) * (x[i] - x[j]) * K[j, i]
    return phi / n, K, h


def step(x, g, eps, lo, hi, h=None):
    """One SVGD update; returns (new particles, phi, h)."""
    phi, _, h = direction(x, g, h)
    return np.clip(np.asarray(x, dtype=np.float64) + eps * phi, lo, hi), phi, h
