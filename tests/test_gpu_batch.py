"""Batched rendering: every scene's outputs from the persistent batch kernels
(graph replay and direct launch) are bitwise those of st_trace on the scene
alone with the same tuning."""
from __future__ import annotations

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu

# batched rendering is switched off in the library (st_batch_create refuses)
DISABLED = pytest.mark.skip(reason="batched rendering is switched off: a batch creation did not return on the "
                                   "device and the cause is not identified; st_batch_create refuses until it is")


def _log(*a):
    print(*a, flush=True)


def _scenes(idx, shrink):
    out = []
    for i in idx:
        sc = sg.config4_scene(i)
        sc.camera.width = max(8, sc.camera.width // shrink)
        sc.camera.height = max(8, sc.camera.height // shrink)
        out.append(sc)
    return out


def _standalone(sc, tuning):
    import torch
    from paper_2304_09673_amd import st
    s = st.Scene(sc)
    s.build_abuffer(sc.camera, tuning)
    d, n, _ = s.trace()
    torch.cuda.synchronize()
    return d.cpu().numpy(), n.cpu().numpy()


@DISABLED
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_batch_equals_standalone(tile):
    import torch
    from paper_2304_09673_amd import st
    scs = _scenes(range(6), 4)
    _log("scenes", [(sc.n_prims, sc.camera.width, sc.camera.height) for sc in scs])
    tune = st.default_tuning(tile=tile, max_new=16)
    ref = [_standalone(sc, tune) for sc in scs]
    _log("standalone done")
    handles = [st.Scene(sc) for sc in scs]
    b = st.Batch(handles, [sc.camera for sc in scs], tuning=tune)
    _log("batch created")
    for use_graph in (False, True, True, True):
        _log("render graph", use_graph)
        for d in b.depths:
            d.fill_(-1.0)
        # eager work between replays
        torch.cuda.synchronize()
        b.render(use_graph=use_graph)
        torch.cuda.synchronize()
        for i, (dr, nr) in enumerate(ref):
            np.testing.assert_array_equal(b.depths[i].cpu().numpy(), dr, err_msg=f"scene {i} graph={use_graph}")
            np.testing.assert_array_equal(b.normals[i].cpu().numpy(), nr, err_msg=f"scene {i} graph={use_graph}")
    stats = b.stats()
    assert all(s["stalled"] == 0 for s in stats)
    assert sum(s["rays"] for s in stats) == sum(sc.camera.width * sc.camera.height for sc in scs)
    b.close()


@DISABLED
def test_batch_with_wide_tiles_equals_standalone():
    """A scene whose tiles overlap more than the LDS fast-path capacity."""
    import torch
    from paper_2304_09673_amd import st
    scs = [sg.config5(width=96, height=64), sg.config1(seed=2, width=64, height=64)]
    tune = st.default_tuning(tile=16, max_new=64, sub_depth=0.25)
    ref = [_standalone(sc, tune) for sc in scs]
    handles = [st.Scene(sc) for sc in scs]
    b = st.Batch(handles, [sc.camera for sc in scs], tuning=tune)
    b.render(use_graph=True)
    torch.cuda.synchronize()
    stats = b.stats()
    assert stats[0]["wide_tiles"] > 0
    for i, (dr, nr) in enumerate(ref):
        np.testing.assert_array_equal(b.depths[i].cpu().numpy(), dr)
        np.testing.assert_array_equal(b.normals[i].cpu().numpy(), nr)
    b.close()


@DISABLED
def test_batch_stale_after_rebuild():
    from paper_2304_09673_amd import st
    scs = _scenes(range(2), 8)
    handles = [st.Scene(sc) for sc in scs]
    b = st.Batch(handles, [sc.camera for sc in scs])
    cam = sg.Camera(width=32, height=32)
    handles[0].build_abuffer(cam)
    with pytest.raises(st.StError):
        b.render()
    b.close()


@DISABLED
def test_batch_rejects_bad_input():
    from paper_2304_09673_amd import st
    sc = sg.config1(seed=0, width=32, height=32)
    h = st.Scene(sc)
    with pytest.raises(st.StError):
        st.Batch([h, h], [sc.camera, sc.camera])
    with pytest.raises(st.StError):
        st.Batch([h], [sc.camera], tuning=st.default_tuning(step_mode=st.ST_STEP_OVERRELAX))


def test_batch_refuses_while_switched_off():
    """The switched-off batch entry points fail loudly (no silent fallback)."""
    from paper_2304_09673_amd import st
    sc = sg.config1(seed=0, width=32, height=32)
    h = st.Scene(sc)
    with pytest.raises(st.StError, match="disabled"):
        st.Batch([h], [sc.camera])
