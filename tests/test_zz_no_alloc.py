"""st_trace_noalloc (the tracing entry point that allocates nothing; its
scratch is one device array of the library) against st_trace, through the C
ABI: bitwise the same depth and normal images and the same counters, on two
calls in a row with the second frame smaller than the first, on the wide
path, and the refusals (frame above the scratch size, stale camera)."""
from __future__ import annotations

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu

COUNTERS = ("rays", "hits", "unconverged", "field_evals", "grad_evals", "steps", "subfrustums", "empty_views",
            "view_nodes", "max_active", "wide_tiles", "stalled")


def _both(sc, tuning):
    import torch
    from paper_2304_09673_amd import st
    s = st.Scene(sc)
    s.build_abuffer(sc.camera, tuning)
    d0, n0, s0 = s.trace()
    H, W = sc.camera.height, sc.camera.width
    d1 = torch.full((H, W), -3.0, device="cuda")
    n1 = torch.full((H, W, 3), -3.0, device="cuda")
    s1 = s.trace_noalloc(d1, n1)
    torch.cuda.synchronize()
    return s, (d0.cpu().numpy(), n0.cpu().numpy(), s0), (d1.cpu().numpy(), n1.cpu().numpy(), s1)


def _same(a, b, label):
    np.testing.assert_array_equal(b[0], a[0], err_msg=label)
    np.testing.assert_array_equal(b[1], a[1], err_msg=label)
    for k in COUNTERS:
        assert a[2][k] == b[2][k], (label, k, a[2][k], b[2][k])


def test_noalloc_equals_trace_on_two_calls_second_smaller():
    from paper_2304_09673_amd import st
    big = sg.config2(0, 512, 512)
    small = sg.config1(1, 128, 96)
    _, a, b = _both(big, st.default_tuning(tile=16))
    print(f"\n[noalloc 512x512] hits {a[2]['hits']} evals {a[2]['field_evals']}", flush=True)
    assert a[2]["hits"] > 1000
    _same(a, b, "512x512")
    _, a, b = _both(small, st.default_tuning(tile=8))
    print(f"[noalloc 128x96] hits {a[2]['hits']} evals {a[2]['field_evals']}", flush=True)
    assert a[2]["hits"] > 100
    _same(a, b, "128x96")


def test_noalloc_wide_path_equals_trace():
    """Capacity 4: tiles above it run on the wide path (slots in LDS)."""
    from paper_2304_09673_amd import st
    sc = sg.config2(0, 256, 256)
    _, a, b = _both(sc, st.default_tuning(max_active=4))
    assert a[2]["wide_tiles"] > 0
    _same(a, b, "wide")


def test_noalloc_without_stats_and_repeated():
    import torch
    from paper_2304_09673_amd import st
    sc = sg.config1(2, 160, 120)
    s, a, _ = _both(sc, st.default_tuning(tile=32))
    for _ in range(2):
        d = torch.full((120, 160), -3.0, device="cuda")
        n = torch.full((120, 160, 3), -3.0, device="cuda")
        assert s.trace_noalloc(d, n, stats=False) is None
        torch.cuda.synchronize()
        np.testing.assert_array_equal(d.cpu().numpy(), a[0])
        np.testing.assert_array_equal(n.cpu().numpy(), a[1])


def test_noalloc_refuses_frames_above_its_scratch():
    """4096x2816 pixels = 180,224 blocks of 8x8, above the 161,319 records the
    32 MiB scratch holds: ST_E_CAPACITY and nothing written."""
    import torch
    from paper_2304_09673_amd import st
    sc = sg.config1(0, 4096, 2816)
    s = st.Scene(sc)
    s.build_abuffer(sc.camera, st.default_tuning(tile=32))
    d = torch.full((2816, 4096), -3.0, device="cuda")
    n = torch.full((2816, 4096, 3), -3.0, device="cuda")
    with pytest.raises(st.StError) as e:
        s.trace_noalloc(d, n)
    assert e.value.code == st.ST_E_CAPACITY
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((d == -3.0).all()) and bool((n == -3.0).all())


def test_noalloc_rejects_stale_camera():
    import torch
    from paper_2304_09673_amd import st
    sc = sg.config1(0, 64, 64)
    s = st.Scene(sc)
    s.build_abuffer(sc.camera)
    other = sg.Camera(width=64, height=64, eye=(0.0, 0.5, 4.0))
    d = torch.empty((64, 64), device="cuda")
    n = torch.empty((64, 64, 3), device="cuda")
    with pytest.raises(st.StError) as e:
        s.trace_noalloc(d, n, camera=other)
    assert e.value.code == st.ST_E_STALE
