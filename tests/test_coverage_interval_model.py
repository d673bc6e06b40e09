"""A CPU model of the coverage passes' per-line interval (k_count, k_emit): the float steps of
the exact floor divisions, emulated in float32, against the integer coverage predicate tested
pixel by pixel (Sec. 5.2, the strips of the shading pass, on the 1/16-pixel grid).

On a line along a segment's major axis, t_num and the cross product are linear in the minor
pixel index x, so the slab 0 <= t_num < t_den and the strip cross^2 < R^2 t_den each hold on
an interval of x; the kernels intersect them with the segment's box as
x in [-floor((s_max + c) / B), floor((s_max - c) / B)] and the slab's pair of bounds, where
each floor(n / d) is the float quotient n * (1/d) - 2^-16 rounded down, clamped to [-17, 17],
plus one exact integer test.  The model uses reciprocals one ulp either side of the rounded
one (the hardware reciprocal errs by at most one ulp) and covers the extreme magnitudes the
kernels admit (half-widths up to 2048 px, segments up to 1024 px per axis).
"""
import math
import random

import numpy as np

F32 = np.float32


def _rcp(d, ulps):
    r = F32(1.0) / F32(d)
    return np.nextafter(r, F32(np.inf if ulps > 0 else -np.inf), dtype=np.float32) if ulps else r


def _fma_f32(a, b, c):
    # a * b is exact in float64 for two float32 operands; one rounding to float32 after the add
    return float(F32(np.float64(a) * np.float64(b) + np.float64(c)))


def _floordiv_small(n, d, rd, bias=2.0**-16, correct=True):
    assert -2**31 <= n < 2**31
    q = min(max(math.floor(_fma_f32(F32(n), rd, -bias)), -17), 17)
    return q + (1 if correct and q * d + d <= n else 0)


def _line(rng, du, dv, R, eu, ev0, nx, **fd):
    """The kernel's interval and the brute-force set for one line of up to 16 pixels."""
    tden = du * du + dv * dv
    smax = math.isqrt(R * R * tden - 1)
    tn = ev0 * dv + eu * du
    cr = ev0 * du - eu * dv
    assert abs(tn) < 2**31 and abs(cr) < 2**31
    sgu = -1 if du < 0 else 1
    sgv = -1 if dv < 0 else 1
    B, A = 16 * abs(du), 16 * abs(dv)
    cl, tl = sgu * cr, sgv * tn
    lo, hi = (1 - tden, 0) if dv < 0 else (0, tden - 1)
    rB, rA = _rcp(B, rng.choice((-1, 0, 1))), _rcp(max(A, 1), rng.choice((-1, 0, 1)))
    m = smax + 16 * B
    cc = min(max(cl, -m), m)
    x0 = max(0, -_floordiv_small(smax + cc, B, rB, **fd))
    x1 = min(nx, _floordiv_small(smax - cc, B, rB, **fd))
    if A > 0:
        tc = min(max(tl, lo - 16 * A), hi + 1)
        x0 = max(x0, -_floordiv_small(tc - lo, A, rA, **fd))
        x1 = min(x1, _floordiv_small(hi - tc, A, rA, **fd))
    elif tl < lo or tl > hi:
        x1 = -1
    got = list(range(x0, x1 + 1))
    want = []
    for x in range(nx + 1):
        ev = ev0 + 16 * x
        t = ev * dv + eu * du
        c = ev * du - eu * dv
        if 0 <= t < tden and c * c < R * R * tden:
            want.append(x)
    # the emit pass's t_num along the line: the sign of dv times the normalised parameter
    sgn = -1 if lo < 0 else 1
    tnums = [sgn * (tl + x * A) for x in got]
    return got, want, tnums, [(ev0 + 16 * x) * dv + eu * du for x in got]


def test_line_intervals_equal_the_pixel_predicate():
    assert _random_lines(random.Random(20240517), 30000) == 0


def test_the_model_fails_with_a_planted_mistake():
    # a bias on the wrong side, or no exact integer test, adds or misses pixels
    assert _random_lines(random.Random(5), 30000, bias=-2.0**-16) > 0
    assert _random_lines(random.Random(5), 30000, correct=False) > 0


def _random_lines(rng, n, **fd):
    nonempty = bad = 0
    for _ in range(n):
        du = rng.choice((1, -1)) * rng.randint(1, rng.choice((16, 64, 256, 2048, 16384)))
        dv = rng.choice((1, -1)) * rng.randint(0, abs(du))
        r = rng.random()
        if r < 0.05:
            dv = 0
        elif r < 0.1:
            dv = rng.choice((1, -1)) * abs(du)
        R = rng.choice((rng.randint(8, 40), rng.randint(8, 600), rng.randint(8, 32776), 32776))
        lo_u, hi_u = min(0, du) - R, max(0, du) + R
        lo_v, hi_v = min(0, dv) - R, max(0, dv) + R
        if rng.random() < 0.5:   # lines through the strip
            eu = rng.randint(lo_u, hi_u)
            ev0 = int(eu * dv / du) + rng.randint(-R - 16 * 15, R)
        else:                    # the box's corners and edges
            eu = rng.choice((lo_u, hi_u, rng.randint(lo_u, hi_u)))
            ev0 = rng.choice((lo_v, hi_v - 16 * 15, rng.randint(lo_v, hi_v)))
        ev0 = max(lo_v, min(ev0, hi_v))
        nx = rng.randint(0, max(0, min(15, (hi_v - ev0) // 16)))
        got, want, tnums, tnums_direct = _line(rng, du, dv, R, eu, ev0, nx, **fd)
        bad += got != want
        assert got != want or tnums == tnums_direct
        nonempty += bool(want)
    assert nonempty > n // 10
    return bad


def test_line_intervals_at_exact_strip_and_slab_boundaries():
    # lines whose pixel centres sit exactly on the strip edge (cross^2 = R^2 t_den - k) or on
    # the slab's ends (t_num = 0, t_den - 1, t_den)
    rng = random.Random(7)
    hits = 0
    for _ in range(20000):
        du = rng.choice((1, -1)) * rng.randint(1, 400)
        dv = rng.choice((1, -1)) * rng.randint(0, abs(du))
        R = rng.randint(8, 64)
        eu = rng.randint(min(0, du) - R, max(0, du) + R)
        ev0 = int(eu * dv / du) - 16 * rng.randint(0, 15) + rng.randint(-R, R)
        nx = 15
        got, want, _, _ = _line(rng, du, dv, R, eu, ev0, nx)
        assert got == want, (du, dv, R, eu, ev0)
        tden = du * du + dv * dv
        for x in range(nx + 1):
            ev = ev0 + 16 * x
            t = ev * dv + eu * du
            c = ev * du - eu * dv
            if t in (0, tden - 1, tden) or abs(c * c - R * R * tden) <= tden:
                hits += 1
    assert hits > 50
