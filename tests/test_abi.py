"""The C-ABI library loads, exports every symbol include/hair.h declares, and validates its
arguments on the host before any launch (a host-only context, device = -1, reaches the
validation layer without a GPU)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "hair.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hair_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def B():
    from paper_2405_10565_amd import binding
    return binding


def test_library_exports_every_declared_symbol(B):
    declared = _declared_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(B.lib, name), name
    assert sorted(B.EXPORTS) == declared


def test_version_and_error_string(B):
    assert B.lib.hair_version() >= 100
    assert isinstance(B.last_error(), str)


@pytest.fixture()
def hctx(B):
    ctx = B.Context(device=-1)
    yield ctx
    ctx.close()


def _asset(n=4, v=5):
    rng = np.random.default_rng(0)
    xyz = rng.normal(size=(3, n * v)).astype(np.float32) * 0.01
    return n, v, xyz, np.full(n, 8e-5, np.float32), np.full((3, n), 0.5, np.float32)


MAT = (1.55, math.radians(-3.0), 0.3, 0.3)


def test_upload_validation_codes(B, hctx):
    n, v, xyz, w, s = _asset()
    with pytest.raises(B.HairError) as e:
        hctx.upload(n, v, xyz, w, s, MAT)               # valid -> no device
    assert e.value.code == B.HAIR_EDEVICE
    bad = xyz.copy(); bad[1, 3] = np.nan
    for args, code in [
        ((0, v, xyz, w, s, MAT), B.HAIR_EINVAL),
        ((n, 1, xyz, w, s, MAT), B.HAIR_EINVAL),
        ((n, v, bad, w, s, MAT), B.HAIR_EINVAL),
        ((n, v, xyz, np.zeros(n, np.float32), s, MAT), B.HAIR_EINVAL),
        ((n, v, xyz, w, -s, MAT), B.HAIR_EINVAL),
        ((n, v, xyz, w, s, (0.9, 0.0, 0.3, 0.3)), B.HAIR_EINVAL),      # eta <= 1
        ((n, v, xyz, w, s, (1.55, 0.0, 0.0, 0.3)), B.HAIR_EINVAL),     # beta_m = 0
    ]:
        with pytest.raises(B.HairError) as e:
            hctx.upload(*args)
        assert e.value.code == code, args[:2]


def test_rttd_material_validation(B, hctx):
    """R / TT / D materials: valid ones reach the device check, out-of-range widths,
    negative or over-unity attenuations and unknown models are rejected on the host."""
    import dataclasses
    import hairsynth as hs
    n, v, xyz, w, s = _asset()
    good = hs.Material.rttd()
    with pytest.raises(B.HairError) as e:
        hctx.upload(n, v, xyz, w, s, good)
    assert e.value.code == B.HAIR_EDEVICE
    m = B.make_material(good)
    assert m.model == 1 and abs(m.gamma_tt - 0.3) < 1e-7 and list(m.a_d) == pytest.approx([0.3, 0.16, 0.09])
    for change in [dict(beta_r=0.0), dict(beta_tt=2.5), dict(gamma_tt=-0.1), dict(gamma_tt=float("nan")),
                   dict(a_r=(-0.1, 0.1, 0.1)), dict(a_d=(0.8, 0.1, 0.1)), dict(model=2)]:
        with pytest.raises(B.HairError) as e:
            hctx.upload(n, v, xyz, w, s, dataclasses.replace(good, **change))
        assert e.value.code == B.HAIR_EINVAL, change
    # model 1 ignores the R / TT / TRT fields
    with pytest.raises(B.HairError) as e:
        hctx.upload(n, v, xyz, w, s, dataclasses.replace(good, eta=0.5, beta_m=0.0))
    assert e.value.code == B.HAIR_EDEVICE


def test_curved_and_shadowed_validation(B, hctx):
    """Argument checks of the curved and shadowed renders happen on the host, before the
    asset lookup (a host-only context has no assets)."""
    c = _cam(B)
    la, nl = B.make_lights([type("L", (), dict(kind=0, vec=[0, 0, 1], rgb=[1, 1, 1]))()])
    img = C.c_void_p(1)
    for level, mpx, msub in [(0, 4, 16), (1, 0, 16), (1, 4, 0), (1, 4, 17)]:
        assert B.lib.hair_render_curved(hctx.handle, None, 0, level, C.byref(c), la, nl, mpx, msub, img, None,
                                        None) == B.HAIR_EINVAL
    assert B.lib.hair_render_curved(hctx.handle, None, 0, 1, C.byref(c), la, nl, 4, 16, img, None,
                                    None) == B.HAIR_ENOENT
    for r, k, d in [(8, 4, 0.02), (64, 0, 0.02), (64, 8, 0.02), (64, 4, 0.0), (64, 4, float("nan"))]:
        sh = B.hair_shadow(r, k, d)
        assert B.lib.hair_render_shadowed(hctx.handle, None, 0, 0, C.byref(c), la, nl, C.byref(sh), img, None,
                                          None) == B.HAIR_EINVAL
    sh = B.hair_shadow(64, 4, 0.02)
    assert B.lib.hair_render_shadowed(hctx.handle, None, 0, 0, C.byref(c), la, nl, C.byref(sh), img, None,
                                      None) == B.HAIR_ENOENT


def _cam(B, W=64, H=32, **kw):
    c = B.hair_camera()
    c.pos[:] = [0, 0, 1]
    c.rot[:] = [1, 0, 0, 0, 1, 0, 0, 0, 1]
    c.fx = c.fy = 50.0
    c.cx, c.cy = W / 2, H / 2
    c.width, c.height = W, H
    c.z_near = 0.01
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_render_validation_before_lookup(B, hctx):
    la, nl = B.make_lights([type("L", (), dict(kind=0, vec=[0, 0, 1], rgb=[1, 1, 1]))()])
    st = B.hair_stats()
    call = lambda cam, lights=la, n=nl: B.lib.hair_render(hctx.handle, None, 1, 0, C.byref(cam), lights, n,
                                                          C.c_void_p(1), C.c_void_p(0), C.byref(st))
    assert call(_cam(B)) == B.HAIR_ENOENT                       # valid arguments, unknown asset
    assert call(_cam(B, width=0)) == B.HAIR_EINVAL
    assert call(_cam(B, fx=float("nan"))) == B.HAIR_EINVAL
    assert call(_cam(B, z_near=0.0)) == B.HAIR_EINVAL
    assert call(_cam(B), la, 0) == B.HAIR_EINVAL
    assert call(_cam(B), la, B.HAIR_MAX_LIGHTS + 1) == B.HAIR_EINVAL
    bad, _ = B.make_lights([type("L", (), dict(kind=0, vec=[0, 0, 2], rgb=[1, 1, 1]))()])
    assert call(_cam(B), bad, 1) == B.HAIR_EINVAL               # not a unit direction
    bad2, _ = B.make_lights([type("L", (), dict(kind=3, vec=[0, 0, 1], rgb=[1, 1, 1]))()])
    assert call(_cam(B), bad2, 1) == B.HAIR_EINVAL
    assert "kind" in B.last_error()


def test_budget_and_workspace_estimate(B):
    ctx = B.Context(device=-1, budget_bytes=1 << 20)
    assert ctx.memory() == (0, 1 << 20)
    ctx.close()
    e1 = B.ws_estimate(1000, 256, 256)
    e2 = B.ws_estimate(100000, 1920, 1080)
    assert 0 < e1 < e2
    assert B.ws_estimate(10, 16, 16, 10**9) > 4 * 10**9         # pairs dominate when given


def test_null_and_unknown_handles(B, hctx):
    assert B.lib.hair_release(hctx.handle, 77) == B.HAIR_ENOENT
    assert B.lib.hair_ctx_destroy(None) == B.HAIR_EINVAL
    assert B.lib.hair_ws_destroy(None) == B.HAIR_EINVAL
    nl = C.c_int32()
    assert B.lib.hair_lod_info(hctx.handle, 5, C.byref(nl), None, 0, None) == B.HAIR_ENOENT


def test_async_render_validation(B, hctx):
    """hair_render_async needs a workspace of its own context and checks its arguments on the
    host; hair_ws_finish on a workspace that holds no frame returns OK with zeroed stats."""
    la, nl = B.make_lights([type("L", (), dict(kind=0, vec=[0, 0, 1], rgb=[1, 1, 1]))()])
    c = _cam(B)
    img = C.c_void_p(1)
    assert B.lib.hair_render_async(hctx.handle, None, 0, 0, C.byref(c), la, nl, img, None) == B.HAIR_EINVAL
    ws = hctx.workspace()
    assert B.lib.hair_render_async(hctx.handle, ws.handle, 0, 0, C.byref(_cam(B, width=0)), la, nl, img,
                                   None) == B.HAIR_EINVAL
    assert B.lib.hair_render_async(hctx.handle, ws.handle, 0, 0, C.byref(c), la, 0, img, None) == B.HAIR_EINVAL
    assert B.lib.hair_render_async(hctx.handle, ws.handle, 0, 0, C.byref(c), la, nl, None, None) == B.HAIR_EINVAL
    assert B.lib.hair_render_async(hctx.handle, ws.handle, 0, 0, C.byref(c), la, nl, img, None) == B.HAIR_ENOENT
    other = B.Context(device=-1)
    ows = other.workspace()
    assert B.lib.hair_render_async(hctx.handle, ows.handle, 0, 0, C.byref(c), la, nl, img, None) == B.HAIR_EINVAL
    st = B.hair_stats()
    st.fragments = 7
    assert B.lib.hair_ws_finish(ws.handle, C.byref(st)) == B.HAIR_OK and st.fragments == 0
    assert B.lib.hair_ws_finish(None, C.byref(st)) == B.HAIR_EINVAL
    ws.close()
    other.close()
