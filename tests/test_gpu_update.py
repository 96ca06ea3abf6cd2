"""Primitive edits without re-flattening: after st_update_primitives and a
new A-buffer, the images equal those of a scene flattened from the edited
tree, and match the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import scenegen as sg
from gpu_util import all_pixels, compare

pytestmark = pytest.mark.gpu


def _edit(sc, rng, count):
    prims = np.nonzero(np.isin(sc.kind, sg.PRIMITIVE_KINDS))[0]
    ids = rng.choice(prims, size=count, replace=False)
    params = sc.params.copy()
    for i in ids:
        params[i, 0:3] += rng.normal(0, 0.15, 3).astype(np.float32)   # move the centre / first end
        if sc.kind[i] == sg.CAPSULE:
            params[i, 3:6] += rng.normal(0, 0.15, 3).astype(np.float32)
    return ids, params


@pytest.mark.parametrize("which,count", [("c1", 3), ("c2", 20), ("c2", 100)])
def test_update_equals_reflatten(which, count):
    import torch
    from paper_2304_09673_amd import st
    sc = sg.config1(seed=4, width=128, height=128) if which == "c1" else sg.config2(seed=1, width=192, height=192)
    rng = np.random.default_rng(count)
    ids, params = _edit(sc, rng, count)
    tune = st.default_tuning(tile=16)
    s = st.Scene(sc)
    s.build_abuffer(sc.camera, tune)
    s.trace()
    s.update_primitives(ids, sc.kind[ids], params[ids])
    with pytest.raises(st.StError):
        s.trace()                      # A-buffer stale after an edit
    s.build_abuffer(sc.camera, tune)
    d1, n1, _ = s.trace()
    edited = sg.Scene(sc.name + "-edited", sc.kind, sc.left, sc.right, params, sc.root, sc.camera, dict(sc.meta))
    s2 = st.Scene(edited)
    s2.build_abuffer(sc.camera, tune)
    d2, n2, _ = s2.trace()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(d1.cpu().numpy(), d2.cpu().numpy())
    np.testing.assert_array_equal(n1.cpu().numpy(), n2.cpu().numpy())
    assert abs(s.info()["extent"] - s2.info()["extent"]) == 0.0
    px, py = all_pixels(sc.camera)
    r = compare(edited, d1.cpu().numpy(), n1.cpu().numpy(), px[::3], py[::3])
    assert r["fail"] == 0, r


def test_update_rejects_bad_edits_atomically():
    import torch
    from paper_2304_09673_amd import st
    sc = sg.config2(seed=2, width=64, height=64)
    s = st.Scene(sc)
    s.build_abuffer(sc.camera)
    d0, _, _ = s.trace()
    d0 = d0.cpu().numpy()
    prims = np.nonzero(np.isin(sc.kind, sg.PRIMITIVE_KINDS))[0]
    ops = np.nonzero(~np.isin(sc.kind, sg.PRIMITIVE_KINDS))[0]
    good = prims[0]
    two = sc.params[[good, prims[1]]].copy()
    two[1, 6 if sc.kind[prims[1]] == sg.CAPSULE else 3] = -1.0                      # radius / extent < 0
    bad_cases = [
        ([ops[0]], sc.kind[[ops[0]]], sc.params[[ops[0]]]),                       # an operator
        ([good, prims[1]], sc.kind[[good, prims[1]]], two),                         # second entry invalid
        ([len(sc.kind)], [sg.SPHERE], sc.params[[good]]),                           # out of range
    ]
    other = next(k for k in (sg.SPHERE, sg.BOX, sg.CAPSULE) if k != sc.kind[good])
    p_kind = sc.params[[good]].copy()
    p_kind[0, 3:10] = [0.1, 0.1, 0.1, 0.2, 0.2, 0.2, 1.0]
    bad_cases.append(([good], [other], p_kind))                                      # kind changed
    for ids, kinds, params in bad_cases:
        with pytest.raises(st.StError):
            s.update_primitives(ids, kinds, params)
    # nothing changed: the A-buffer is still valid and the image identical
    d1, _, _ = s.trace()
    np.testing.assert_array_equal(d1.cpu().numpy(), d0)
