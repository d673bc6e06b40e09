"""Writes the stored expected values of the full-size GPU parity tests from the oracle alone.

    python tests/golden/make_golden.py [case ...]      # all cases when none is named

Each case is a seeded synthetic frame (hairsynth generator) rendered by the oracle's
rasterisation (oracle.render.rasterize, in row bands to bound memory).  Stored per case:
the frame's fragment count, the count of every image row, and the deepest pixels (most
fragments) with their counts.  Nothing here calls the HIP library.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import hairsynth as hs  # noqa: E402
from oracle import lod as OL  # noqa: E402
from oracle import mixed as M  # noqa: E402
from oracle import render as R  # noqa: E402


def strands_100k_1080p():
    """100k strands x 32 segments at 1920x1080 (the benchmark's frame)."""
    asset, cam, _ = hs.config(2)
    return R.strand_level(asset), cam


def mixed_20k_1080p():
    """20k strands x 16 segments with 2000 / 300 / 40 thick hairs, a seeded random level per
    group and segment, at 1920x1080."""
    asset = hs.make_asset(20000, 16, 90.0, seed=35, sigma_spread=True)
    assigns = hs.kmeans_hierarchy(asset, (2000, 300, 40), seed=35)
    lods = [OL.build_level(asset, a) for a in assigns]
    geoms = M.level_geoms(asset, lods)
    grps = M.groups(assigns)
    G, S = int(assigns[-1].max()) + 1, asset.segs
    levels = np.random.default_rng(35).integers(0, 4, size=(G, S)).astype(np.int32)
    return M.mixed_geometry(geoms, grps, levels), hs.camera_for(asset, 1920, 1080)


CASES = {"strands_100k_1080p": strands_100k_1080p, "mixed_20k_1080p": mixed_20k_1080p}


def fragment_census(geom, cam, band: int = 24, top: int = 4) -> dict:
    W, H = cam.width, cam.height
    rows = np.zeros(H, dtype=np.int64)
    deep = []
    for y0 in range(0, H, band):
        h = min(band, H - y0)
        ras = R.rasterize(geom, cam, rect=(0, y0, W, h))
        y = ras.pix // W
        rows[y0:y0 + h] = np.bincount(y - y0, minlength=h)[:h]
        cnt = np.bincount(ras.pix - y0 * W, minlength=W * h)
        for p in np.argsort(-cnt, kind="stable")[:top]:
            deep.append((int(cnt[p]), int(p % W), int(y0 + p // W)))
    deep.sort(key=lambda t: (-t[0], t[2], t[1]))
    return {"fragments": int(rows.sum()), "rows": rows.tolist(),
            "deepest": [{"x": x, "y": y, "count": c} for c, x, y in deep[:top]]}


def main(names):
    for name in names or sorted(CASES):
        geom, cam = CASES[name]()
        out = fragment_census(geom, cam)
        out["case"] = CASES[name].__doc__.strip().split("\n")[0]
        path = os.path.join(HERE, f"{name}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"{name}: {out['fragments']} fragments -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
