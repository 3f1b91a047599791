"""Particle detection on a reconstructed volume (CPU, test utility).

TEST INFRASTRUCTURE ONLY.  Used by the recovery and centroid tests; the
product path never imports it.

Paper, section "Methodology" (segmentation) and "Synthetic Turbulent Flow":
  * keep voxels above a small fraction (1/256 by default) of the maximum;
  * connected components (26-connectivity, which the paper leaves unstated);
  * drop components smaller than the minimum object volume (5 voxels);
  * particle position = intensity-weighted centroid of the component;
  * match to ground truth by nearest neighbour.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

__all__ = ["detect", "match"]


def detect(x: np.ndarray, rel_threshold: float = 1.0 / 256.0, min_voxels: int = 5):
    """Return centroids [n][3] (z, y, x) of the segmented objects."""
    x = np.asarray(x, dtype=np.float64)
    if x.size == 0 or x.max() <= 0:
        return np.zeros((0, 3))
    mask = x > rel_threshold * x.max()
    labels, n = ndimage.label(mask, structure=np.ones((3, 3, 3), dtype=bool))
    if n == 0:
        return np.zeros((0, 3))
    idx = np.arange(1, n + 1)
    sizes = ndimage.sum_labels(np.ones_like(x), labels, idx)
    keep = idx[sizes >= min_voxels]
    if len(keep) == 0:
        return np.zeros((0, 3))
    cents = ndimage.center_of_mass(np.where(mask, x, 0.0), labels, keep)
    return np.asarray(cents, dtype=np.float64).reshape(-1, 3)


def match(found: np.ndarray, truth: np.ndarray, max_dist: float = 2.0):
    """Greedy nearest-neighbour matching; returns (pairs [(i_truth, i_found)], errors [n][3])."""
    found = np.asarray(found, dtype=np.float64).reshape(-1, 3)
    truth = np.asarray(truth, dtype=np.float64).reshape(-1, 3)
    if len(found) == 0 or len(truth) == 0:
        return [], np.zeros((0, 3))
    d = np.linalg.norm(truth[:, None, :] - found[None, :, :], axis=2)
    pairs, errs = [], []
    used_t, used_f = set(), set()
    for flat in np.argsort(d, axis=None):
        i, j = np.unravel_index(flat, d.shape)
        if d[i, j] > max_dist:
            break
        if i in used_t or j in used_f:
            continue
        used_t.add(i)
        used_f.add(j)
        pairs.append((int(i), int(j)))
        errs.append(found[j] - truth[i])
    return pairs, np.asarray(errs).reshape(-1, 3)
