"""Counts the algorithmic operations per fragment of the shading pass by running the oracle's
definition under an operation counter, and writes tests/golden/ops_per_fragment.json.

    python tests/golden/count_ops.py

What is counted: every elementwise arithmetic operation the oracle's per-fragment path
performs on its float64 tensors (torch) with an input that differs between fragments,
weighted by the number of elements it produces (reductions by inputs minus outputs), divided
by the number of fragments.  Operations on values every fragment shares (material, light and
quadrature-node constants) are computed once per frame and not counted.  The path is the
one the shading kernel executes per fragment: alpha and h (oracle.render.fragment_alpha_h),
the world point and tangent (shading_inputs), the frame (frame), then per light its
direction and irradiance (light_dirs) and the scattering function (f_single for strands,
f_ours with the chord and hair counts for thick hairs), and the front-to-back blend
(composite).  Classes:
  * ops:   add, sub, mul, div, neg, abs, sign, min, max, clamp bounds, select, compare,
           logical, floor/round/remainder, square; a dot product of n terms is n mul + n-1 add
  * trans: exp, log, sqrt, sin, cos, tanh, asin, acos, atan, atan2, erf, sigmoid: one each
The thick hairs' hemisphere terms evaluate an integrand even in h at 8 symmetric
Gauss-Legendre nodes; they count at half weight (an evaluation at 4 nodes is the same rule).
The per-pixel depth sort is not a tensor operation in the oracle (a lexicographic sort); its
cost is taken as ceil(log2 k) compares per fragment for k fragments per pixel, and stored
beside the counts.  The coverage test and the depth key (integer, numpy) belong to the
coverage kernels and are counted separately, per candidate pixel, from oracle.raster.coverage
and depth_key.  Nothing here calls the HIP library.
"""
from __future__ import annotations

import json
import math
import os
import sys
from collections import Counter

import numpy as np
import torch
from torch.overrides import TorchFunctionMode

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import hairsynth as hs  # noqa: E402
from oracle import aggregate as AG  # noqa: E402
from oracle import lod as OL  # noqa: E402
from oracle import render as R  # noqa: E402

ELEM_OPS = {"add", "sub", "mul", "div", "true_divide", "neg", "abs", "sign", "minimum", "maximum", "where",
            "lt", "gt", "le", "ge", "eq", "ne", "logical_and", "logical_or", "logical_not", "bitwise_and",
            "bitwise_or", "bitwise_not", "floor", "ceil", "round", "remainder", "fmod", "square", "rsub",
            "reciprocal", "__add__", "__radd__", "__iadd__", "__sub__", "__rsub__", "__isub__", "__mul__",
            "__rmul__", "__imul__", "__truediv__", "__rtruediv__", "__itruediv__", "__neg__", "__abs__",
            "__lt__", "__gt__", "__le__", "__ge__", "__eq__", "__ne__", "__and__", "__or__", "__invert__",
            "__xor__", "__mod__", "__rmod__", "__floordiv__", "__rdiv__", "__div__"}
TRANS = {"exp", "log", "sqrt", "rsqrt", "sin", "cos", "tan", "tanh", "asin", "arcsin", "acos", "atan", "atan2",
         "arctan2", "erf", "sigmoid", "exp2", "log2", "expm1", "log1p"}
NO_ARITH = {"__getitem__", "__setitem__", "expand", "expand_as", "reshape", "view", "as_tensor", "tensor",
            "full_like", "zeros_like", "ones_like", "zeros", "ones", "full", "cat", "stack", "numpy", "item",
            "dim", "size", "clone", "to", "detach", "__len__", "__format__", "__bool__", "__float__", "__int__",
            "repeat_interleave", "index_select", "unsqueeze", "squeeze", "contiguous", "arange", "__index__",
            "argmin", "index_copy", "any", "all", "__get__", "shape", "dtype", "device", "__repr__", "float",
            "double", "long", "int", "bool", "type", "numel", "requires_grad_", "tolist", "copy_", "nonzero",
            "__array__", "max", "min", "t", "T", "transpose", "flatten", "__iter__", "__contains__", "split",
            "new_zeros", "new_ones", "new_full", "fill_", "empty_like", "is_floating_point", "element_size"}


def _numel(x):
    return x.numel() if isinstance(x, torch.Tensor) else 1


def _varying(x, F):
    """Whether tensor x holds different values for different fragments (dimension 0 of
    length F); values shared by every fragment (material, light and quadrature constants,
    expanded or not) are computed once per frame, not per fragment."""
    if not isinstance(x, torch.Tensor) or x.dim() == 0 or x.shape[0] != F or F <= 1:
        return False
    if x.stride(0) == 0:
        return False
    return not bool((x == x[:1]).all())


class OpCounter(TorchFunctionMode):
    """Counts arithmetic on tensors (elements produced per operation)."""

    def __init__(self, F, shared_filter=True):
        super().__init__()
        self.F = F
        self.shared_filter = shared_filter
        self.ops = 0
        self.trans = 0
        self.unknown = Counter()

    def __torch_function__(self, func, types, args=(), kwargs=None):
        kwargs = kwargs or {}
        out = func(*args, **kwargs)
        name = getattr(func, "__name__", "") or str(func)
        name = name.split(".")[-1]
        n = _numel(out[0] if isinstance(out, tuple) else out)
        ins = [a for a in list(args) + list(kwargs.values()) if isinstance(a, torch.Tensor)]
        for a in args:
            if isinstance(a, (list, tuple)):
                ins += [b for b in a if isinstance(b, torch.Tensor)]
        if self.shared_filter and name not in NO_ARITH and not any(_varying(a, self.F) for a in ins):
            return out                                                # the same for every fragment
        if name in ELEM_OPS:
            self.ops += n
        elif name in ("__pow__", "pow") and len(args) > 1 and isinstance(args[1], (int, float)) and args[1] == 2:
            self.ops += n
        elif name in ("__pow__", "pow", "__rpow__"):
            self.trans += 2 * n                                     # exp(b log a)
            self.ops += n
        elif name in TRANS:
            self.trans += n
        elif name == "clamp":
            bounds = sum(1 for k in ("min", "max") if kwargs.get(k) is not None) + max(0, len(args) - 1)
            self.ops += n * max(1, min(bounds, 2))
        elif name in ("sum", "index_add"):
            src = args[0] if name == "sum" else args[3]
            self.ops += _numel(src) - (n if name == "sum" else 0)
        elif name == "mean":
            self.ops += _numel(args[0])                              # n - 1 adds and a divide per output
        elif name in ("linalg_norm", "norm"):
            x = args[0]
            self.ops += 2 * _numel(x) - n
            self.trans += n
        elif name in ("linalg_cross", "cross"):
            self.ops += 3 * n
        elif name not in NO_ARITH:
            self.unknown[name] += n
        return out


class _HalfWeight:
    """The hemisphere albedos and variances integrate an integrand even in h (the attenuation
    depends on h only through cos gamma_o and cos gamma_t, the front mass through |Phi(p, h)|
    up to a multiple of 2 pi), so the 8-node Gauss-Legendre rule over symmetric nodes is an
    evaluation at 4 of them: hemisphere_stats counts at half weight."""

    def __init__(self, counter, fn):
        self.c = counter
        self.orig = fn

    def __call__(self, *args, **kwargs):
        o0, t0 = self.c.ops, self.c.trans
        out = self.orig(*args, **kwargs)
        self.c.ops -= (self.c.ops - o0) // 2
        self.c.trans -= (self.c.trans - t0) // 2
        return out


def _counted(geom, ras, cam, lights, mat):
    with OpCounter(len(ras.seg)) as c:
        AG.hemisphere_stats = _HalfWeight(c, AG.hemisphere_stats)
        try:
            R.fragment_radiance(geom, ras, cam, lights, mat)
        finally:
            AG.hemisphere_stats = AG.hemisphere_stats.orig
    return c


def count(geom, cam, lights, mat, band):
    """(ops, trans) per fragment of: base (alpha, h, world point, frame), each light, blend."""
    ras = R.rasterize(geom, cam, rect=band)
    F = len(ras.seg)
    res = {"fragments": F}
    c = _counted(geom, ras, cam, [], mat)
    res["base"] = (c.ops / F, c.trans / F)
    unknown = Counter(c.unknown)
    for li, light in enumerate(lights):
        c = _counted(geom, ras, cam, [light], mat)
        res[f"light{li}_kind{light.kind}"] = (c.ops / F - res["base"][0], c.trans / F - res["base"][1])
        unknown.update(c.unknown)
    alpha, L = R.fragment_radiance(geom, ras, cam, lights, mat)
    with OpCounter(F, shared_filter=False) as c:       # (its tensors are per pixel rank, all varying)
        R.composite(ras, alpha, L)
    # (less the image's 1 - T for every pixel, which is per pixel, not per fragment)
    res["blend"] = ((c.ops - ras.W * ras.H) / F, c.trans / F)
    k = np.bincount(ras.pix)
    k = k[k > 0]
    res["sort_compares"] = float(np.sum(k * np.ceil(np.log2(np.maximum(k, 2)))) / F)
    res["unknown"] = dict(unknown)
    return res


NP_TRANS = {"sqrt", "exp", "exp2", "log", "log2", "sin", "cos", "arcsin", "arctan2", "arctan", "tanh"}
NP_FREE = {"astype", "stack", "zeros", "zeros_like", "concatenate", "copy", "reshape", "asarray", "array"}


class _NpCounted(np.ndarray):
    """An array whose elementwise arithmetic (numpy ufuncs, where, clip) is counted by the
    elements it produces, with the same classes as OpCounter; gathers (indexing) and
    conversions are free, as they are there."""
    counter = None

    def __array_ufunc__(self, ufunc, method, *inputs, **kwargs):
        args = [np.asarray(x) if isinstance(x, _NpCounted) else x for x in inputs]
        if "out" in kwargs:
            kwargs["out"] = tuple(np.asarray(x) if isinstance(x, _NpCounted) else x for x in kwargs["out"])
        out = getattr(ufunc, method)(*args, **kwargs)
        c = _NpCounted.counter
        n = int(np.size(out[0] if isinstance(out, tuple) else out))
        if ufunc.__name__ in NP_TRANS:
            c.trans += n
        else:
            c.ops += n
        return np.asarray(out).view(_NpCounted) if isinstance(out, np.ndarray) else out

    def __array_function__(self, func, types, args, kwargs):
        plain = lambda a: np.asarray(a) if isinstance(a, _NpCounted) else a
        args2 = [plain(a) if not isinstance(a, (list, tuple)) else type(a)(plain(b) for b in a) for a in args]
        kwargs2 = {k: plain(v) for k, v in kwargs.items()}
        out = func(*args2, **kwargs2)
        c = _NpCounted.counter
        n = int(np.size(out)) if isinstance(out, np.ndarray) else 0
        if func.__name__ == "where":
            c.ops += n
        elif func.__name__ == "clip":
            c.ops += 2 * n
        elif func.__name__ not in NP_FREE:
            c.unknown[func.__name__] += n
        return out.view(_NpCounted) if isinstance(out, np.ndarray) else out


def _counted_lookup(geom, ras, cam, doms):
    """Operations of the deep opacity map lookup of every fragment: its world point on the
    centre line (oracle.shadow.lookup_point) and, per map, the bilinear, layer-interpolated
    count (dom_count); the maps themselves are the shadow pass's, built outside."""
    from oracle import shadow as SH
    c = OpCounter(len(ras.seg))
    _NpCounted.counter = c
    counted = lambda a: np.asarray(a).view(_NpCounted)
    rv = R.Raster(**{k: (counted(v) if k in ("t_num", "t_den", "izA", "izB") else v)
                     for k, v in vars(ras).items()})
    gv = R.LevelGeom(**{k: (counted(v) if k in ("pA", "pB") else v) for k, v in vars(geom).items()})
    x = SH.lookup_point(gv, rv, cam)
    for dom in doms:
        SH.dom_count(dom, np.asarray(x).view(_NpCounted))
    _NpCounted.counter = None
    return c


def count_shadowed(geom, cam, lights, mat, band, shadow):
    """(ops, trans) per fragment of the shadowed shading pass: base, the map lookup (point and
    per directional light), each light with the hairs in front as the frame has them (a
    strand with n_s > 0 takes the aggregated model, the others the single-fibre one: the
    average over the band's fragments), blend and sort."""
    from oracle import shadow as SH
    res = count(geom, cam, [], mat, band)
    ras = R.rasterize(geom, cam, rect=band)
    F = len(ras.seg)
    Rm, K, delta = shadow
    doms = [SH.build_dom(geom, l.vec, Rm, K, delta) for l in lights if l.kind == 0]
    x = SH.lookup_point(geom, ras, cam)
    ns, it = [], iter(doms)
    for l in lights:
        ns.append(None if l.kind != 0 else torch.as_tensor(SH.dom_count(next(it), x), dtype=torch.float64))
    c = _counted_lookup(geom, ras, cam, doms)
    res["lookup"] = (c.ops / F, c.trans / F)
    res["shadowed_fraction"] = [None if n is None else float((n > 0).double().mean()) for n in ns]
    unknown = Counter(res["unknown"])
    unknown.update(c.unknown)
    base = res["base"]
    for li, light in enumerate(lights):
        single = _counted(geom, ras, cam, [light], mat)
        one = (single.ops / F - base[0], single.trans / F - base[1])
        key = f"light{li}_kind{light.kind}"
        if ns[li] is None:
            res[key] = one
            continue
        # the oracle evaluates both models for every fragment and selects; a fragment takes
        # one of them, so a fragment with hairs in front costs (both - f_single) and one
        # without costs f_single
        with OpCounter(F) as c:
            AG.hemisphere_stats = _HalfWeight(c, AG.hemisphere_stats)
            try:
                R.fragment_radiance(geom, ras, cam, [light], mat, shadow=[ns[li]])
            finally:
                AG.hemisphere_stats = AG.hemisphere_stats.orig
        both = (c.ops / F - base[0], c.trans / F - base[1])
        ours = (both[0] - one[0], both[1] - one[1])
        fr = res["shadowed_fraction"][li]
        res[key] = (fr * ours[0] + (1 - fr) * one[0], fr * ours[1] + (1 - fr) * one[1])
        res[key + "_models"] = {"f_single": one, "f_ours_with_selection": ours}
        unknown.update(c.unknown)
        unknown.update(single.unknown)
    res["unknown"] = dict(unknown)
    return res


def coverage_ops():
    """Integer operations per candidate (pixel, segment) of the coverage predicate, and float32
    operations of the depth key per fragment, from oracle.raster (numpy) by reading: the
    predicate d, e (4 sub), t_num, t_den, cross (6 mul + 3 add/sub), R = hw + 8 (1), the slab
    test (2 compares), cross^2 and R^2 t_den (3 mul) and the compare (1): 20; the key: t = e.d
    / d.d as floats (1 div + 2 conversions), iz = izA + t (izB - izA) (3), the key (1): 7."""
    return {"coverage_per_candidate": 20, "key_per_fragment": 7}


def main():
    out = {"note": __doc__.strip().split("\n")[0]}
    asset, cam, lights = hs.config(2)
    mat = tuple(float(v) for v in asset.material.as_array())
    band = (0, 536, cam.width, 4)
    out["strand_100k_1080p"] = count(R.strand_level(asset), cam, lights, mat, band)
    # a thick-hair level of the same kind as the level sweep's (1k thick hairs from 150k
    # strands x 64 segments), on a smaller groom so the count runs in seconds
    small = hs.make_asset(15000, 64, 90.0, seed=1003, sigma_spread=True)
    lod = OL.build_level(small, hs.kmeans_assign(small, 100, seed=1003))
    cam3 = hs.camera_for(small, 1920, 1080)
    lights3 = hs.default_lights(small, with_point=True)
    out["thick_1080p"] = count(R.cluster_level(lod), cam3, lights3, mat, (0, 536, cam3.width, 4))
    # the shadowed headline frame (deep opacity map 1024^2, 4 layers of 2 cm)
    out["strand_shadowed_100k_1080p"] = count_shadowed(R.strand_level(asset), cam, lights, mat, band, (1024, 4, 0.02))
    out["coverage"] = coverage_ops()
    path = os.path.join(HERE, "ops_per_fragment.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
