"""Per-group, per-segment level of detail and mixed-level frames (oracle; test infrastructure).

Hierarchy (Sec. 5.1, stage 2): the levels are nested, every thick hair of a finer level lies
inside one thick hair of the coarsest level; those coarsest clusters are the groups g.  Level 0
is the strands, levels 1..n the thick-hair levels from finer to coarser.

A frame chooses a level L(g, k) for every group g and segment index k (the paper selects per
cluster of its coarsest level and per segment, Sec. 5.1 step 5) and renders, for each (g, k),
the k-th segments of the owners (strands or thick hairs) of level L(g, k) inside g; rows are
ordered by g, then k, then owner id, and that row index breaks depth ties.

Width of (g, k) at level l: the largest 2 hw (float32, the frame's own half-width) over the
visible k-th segments of level l's owners in g, 0 when none is visible.
  * Initial level (Sec. 5.1 step 5, eps_w of Sec. 6): the coarsest l >= 1 whose width is at
    most eps_w; 0 when no level qualifies.
  * Deferred update (Sec. 5.2, eq. lod_select), in this indexing where larger is coarser:
    from the frame's level L with width w and the width w_c one level coarser, the next level
    is L - 1 (not below 0) when w > eps_w, L + 1 when L < n and w_c <= eps_w, else L.
"""
from __future__ import annotations

import numpy as np

from . import render as R


def groups(assigns):
    """Group of every owner per level (list: level 0 = strands, then each cluster level),
    from the dense assignments of the levels finer -> coarser.  Raises if not nested."""
    top = np.asarray(assigns[-1], dtype=np.int64)
    out = [top.copy()]
    for a in assigns:
        a = np.asarray(a, dtype=np.int64)
        K = int(a.max()) + 1
        g = np.full(K, -1, dtype=np.int64)
        for s in range(a.size):
            if g[a[s]] < 0:
                g[a[s]] = top[s]
            elif g[a[s]] != top[s]:
                raise ValueError("levels are not nested")
        out.append(g)
    return out


def owners_by_group(group_of_owner, G):
    """Owner ids of each group, ascending: list of arrays."""
    order = np.lexsort((np.arange(group_of_owner.size), group_of_owner))
    cuts = np.searchsorted(group_of_owner[order], np.arange(G + 1))
    return [order[cuts[g]:cuts[g + 1]] for g in range(G)]


def level_geoms(asset, lods):
    return [R.strand_level(asset)] + [R.cluster_level(lod) for lod in lods]


def level_widths(geom, grp, G, S, cam):
    """[G, S] float32 widths of one level."""
    _, _, _, _, _, _, _, hw, _, vis = R.segment_records(geom, cam)
    w = np.where(vis, np.float32(2.0) * hw, np.float32(0.0)).reshape(-1, S)
    out = np.zeros((G, S), dtype=np.float32)
    for o in range(w.shape[0]):
        out[grp[o]] = np.maximum(out[grp[o]], w[o])
    return out


def init_levels(geoms, grps, cam, eps_w):
    G, S = int(grps[0].max()) + 1, int(geoms[0].pA.shape[1] // grps[0].size)
    n = len(geoms) - 1
    lev = np.zeros((G, S), dtype=np.int32)
    done = np.zeros((G, S), dtype=bool)
    for l in range(n, 0, -1):
        ok = (level_widths(geoms[l], grps[l], G, S, cam) <= eps_w) & ~done
        lev[ok] = l
        done |= ok
    return lev


def update_levels(geoms, grps, cam, eps_w, levels):
    G, S = levels.shape
    n = len(geoms) - 1
    widths = [level_widths(geoms[l], grps[l], G, S, cam) for l in range(n + 1)]
    nxt = levels.copy()
    for g in range(G):
        for k in range(S):
            L = int(levels[g, k])
            if widths[L][g, k] > eps_w:
                nxt[g, k] = max(L - 1, 0)
            elif L < n and widths[L + 1][g, k] <= eps_w:
                nxt[g, k] = L + 1
    return nxt


def mixed_geometry(geoms, grps, levels) -> R.LevelGeom:
    """Rows of a mixed frame in (g, k, owner) order."""
    G, S = levels.shape
    lists = [owners_by_group(grps[l], G) for l in range(len(geoms))]
    src_level, src_row = [], []
    for g in range(G):
        for k in range(S):
            L = int(levels[g, k])
            own = lists[L][g]
            src_level.append(np.full(own.size, L))
            src_row.append(own * S + k)
    lvl = np.concatenate(src_level) if src_level else np.zeros(0, np.int64)
    row = np.concatenate(src_row) if src_row else np.zeros(0, np.int64)
    n = lvl.size
    pA = np.zeros((3, n), np.float32)
    pB = np.zeros((3, n), np.float32)
    sig = np.zeros((n, 3), np.float32)
    width = np.ones(n, np.float32)
    ahat = np.tile(np.array([[1.0], [0.0], [0.0]], np.float32), (1, n))
    a_len = np.ones(n, np.float32)
    b_len = np.ones(n, np.float32)
    n_total = np.ones(n, np.int32)
    r = np.ones(n, np.float32)
    for l, gm in enumerate(geoms):
        m = lvl == l
        if not m.any():
            continue
        rr = row[m]
        pA[:, m] = gm.pA[:, rr]
        pB[:, m] = gm.pB[:, rr]
        sig[m] = gm.sigma_a[rr]
        if gm.kind == "strand":
            width[m] = gm.width[rr]
        else:
            ahat[:, m] = gm.ahat[:, rr]
            a_len[m], b_len[m] = gm.a_len[rr], gm.b_len[rr]
            n_total[m], r[m] = gm.n_total[rr], gm.r[rr]
    return R.LevelGeom("mixed", pA, pB, sig, width=width, ahat=ahat, a_len=a_len, b_len=b_len, n_total=n_total,
                       r=r, thick=lvl > 0)
