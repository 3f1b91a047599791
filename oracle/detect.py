"""Particle detection on a reconstructed volume (CPU, test utility).

TEST INFRASTRUCTURE ONLY.  Used by the recovery and centroid tests; the
product path never imports it.

Paper, section "Methodology" (segmentation) and "Synthetic Turbulent Flow":
  * keep voxels above a small fraction (1/256 by default) of the maximum;
  * connected components (26-connectivity, which the paper leaves unstated);
  * drop components smaller than the minimum object volume (5 voxels);
  * particle position = intensity-weighted centroid of the component;
  * match to ground truth by nearest neighbour;
  * link particles of successive frames by the method of Crocker & Grier
    (minimum total squared displacement within each subnetwork of candidate
    links closer than the maximum displacement) into tracks, keeping tracks of
    a minimum duration.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

__all__ = ["detect", "match", "objects", "link", "track"]


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


# ----------------------------------------------------------------------------
# Object table and Crocker-Grier linking (section "Synthetic Turbulent Flow":
# weighted centroids of the connected components, tracked by the method of
# Crocker & Grier with a maximum displacement per frame and a minimum track
# duration).
# ----------------------------------------------------------------------------
def objects(x: np.ndarray, rel_threshold: float = 1.0 / 256.0, min_voxels: int = 5):
    """Kept objects, ordered by their smallest linear voxel index, as rows
    (z, y, x, intensity sum, voxel count, smallest linear index); and the
    number of components before the minimum-volume filter."""
    x = np.asarray(x, dtype=np.float64)
    if x.size == 0 or x.max() <= 0:
        return np.zeros((0, 6)), 0
    mask = x > rel_threshold * x.max()
    labels, n = ndimage.label(mask, structure=np.ones((3, 3, 3), dtype=bool))
    if n == 0:
        return np.zeros((0, 6)), 0
    flat = labels.ravel()
    # first occurrence of each label in raster order = its smallest linear index;
    # ndimage numbers labels in that order
    first = np.full(n + 1, -1, dtype=np.int64)
    nz_idx = np.flatnonzero(flat)
    lab = flat[nz_idx]
    order = np.argsort(lab, kind="stable")
    lab_sorted = lab[order]
    starts = np.searchsorted(lab_sorted, np.arange(1, n + 1))
    first[1:] = nz_idx[order][starts]
    idx = np.arange(1, n + 1)
    sizes = ndimage.sum_labels(np.ones_like(x), labels, idx)
    w = np.where(mask, x, 0.0)
    wsum = ndimage.sum_labels(w, labels, idx)
    cents = np.asarray(ndimage.center_of_mass(w, labels, idx), dtype=np.float64).reshape(-1, 3)
    rows = np.column_stack([cents, wsum, sizes, first[1:]])
    return rows[sizes >= min_voxels], n


def _subnetworks(cands, n0):
    """Connected components of the bipartite candidate graph, as lists of
    sources (ascending), each with its candidate targets."""
    parent = list(range(n0))

    def find(a):
        while parent[a] != a:
            a = parent[a]
        return a
    owner = {}
    for i in range(n0):
        for j, _ in cands[i]:
            if j in owner:
                a, b = find(i), find(owner[j])
                if a != b:
                    parent[max(a, b)] = min(a, b)
            else:
                owner[j] = i
    groups = {}
    for i in range(n0):
        if cands[i]:
            groups.setdefault(find(i), []).append(i)
    return [groups[k] for k in sorted(groups)]


def link(prev: np.ndarray, cur: np.ndarray, max_disp: float, spacing=(1.0, 1.0, 1.0), max_subnet: int = 8):
    """Crocker-Grier linking of two frames of positions (z, y, x in voxels;
    spacing converts to physical units).  A candidate link joins a particle of
    `prev` to one of `cur` within max_disp.  Within each subnetwork (a
    connected group of candidate links) the chosen links minimise
    sum(d^2) + max_disp^2 * (number of unlinked particles of prev), each
    particle linked at most once.  Returns link[i] = index in cur or -1.

    Enumeration order (which decides between equal costs): sources in
    ascending index; each takes its candidates by increasing distance (then
    index), "unlinked" last; the first assignment reaching the minimum is
    kept.  Subnetworks of more than max_subnet sources raise ValueError."""
    prev = np.asarray(prev, dtype=np.float64).reshape(-1, 3)
    cur = np.asarray(cur, dtype=np.float64).reshape(-1, 3)
    sp = np.asarray(spacing, dtype=np.float64)
    r2 = float(max_disp) * float(max_disp)
    n0 = len(prev)
    cands = []
    for i in range(n0):
        c = []
        for j in range(len(cur)):
            dz = (cur[j, 0] - prev[i, 0]) * sp[0]
            dy = (cur[j, 1] - prev[i, 1]) * sp[1]
            dx = (cur[j, 2] - prev[i, 2]) * sp[2]
            d2 = dz * dz + dy * dy + dx * dx
            if d2 <= r2:
                c.append((j, d2))
        c.sort(key=lambda t: (t[1], t[0]))
        cands.append(c)
    out = np.full(n0, -1, dtype=np.int64)
    for group in _subnetworks(cands, n0):
        if len(group) > max_subnet:
            raise ValueError(f"subnetwork of {len(group)} particles exceeds {max_subnet}")
        best = [np.inf, None]
        choice = [-1] * len(group)

        def search(k, used, cost):
            if cost >= best[0]:
                return
            if k == len(group):
                best[0], best[1] = cost, list(choice)
                return
            for j, d2 in cands[group[k]]:
                if j not in used:
                    choice[k] = j
                    search(k + 1, used | {j}, cost + d2)
            choice[k] = -1
            search(k + 1, used, cost + r2)
        search(0, frozenset(), 0.0)
        for i, j in zip(group, best[1]):
            out[i] = j
    return out


def track(frames, max_disp: float, spacing=(1.0, 1.0, 1.0), min_len: int = 1):
    """Track ids of every particle of a sequence of frames (lists of positions):
    frame 0 opens tracks 0..n0-1; in each later frame a linked particle keeps
    its source's id and the others open new ids in ascending particle order.
    Returns (ids per frame, track lengths, kept: tracks of at least min_len
    frames)."""
    ids = [np.arange(len(frames[0]), dtype=np.int64)] if len(frames) else []
    nxt = len(frames[0]) if len(frames) else 0
    for t in range(1, len(frames)):
        lk = link(frames[t - 1], frames[t], max_disp, spacing)
        cur = np.full(len(frames[t]), -1, dtype=np.int64)
        for i, j in enumerate(lk):
            if j >= 0:
                cur[j] = ids[t - 1][i]
        for j in range(len(cur)):
            if cur[j] < 0:
                cur[j] = nxt
                nxt += 1
        ids.append(cur)
    lengths = np.zeros(nxt, dtype=np.int64)
    for a in ids:
        np.add.at(lengths, a, 1)
    return ids, lengths, lengths >= min_len
