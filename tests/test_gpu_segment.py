"""Segment tracing (ST_STEP_SEGMENT) on the pruned views: the same parity
rules against the FP64 oracle as the plain tracer, the same hit masks, and no
more stepping evaluations than the plain tracer (its step is never shorter
than the plain safe step)."""
from __future__ import annotations

import numpy as np
import pytest

import scenegen as sg
from gpu_util import all_pixels, assert_masks_agree, compare, gpu_render, stratified_pixels

pytestmark = pytest.mark.gpu


def _report(name, r):
    print(f"\n[{name}] " + " ".join(f"{k}={v}" for k, v in r.items() if k != "fail_idx"), flush=True)


def _pair(sc, **kw):
    from paper_2304_09673_amd import st
    _, d_p, n_p, s_p = gpu_render(sc, st.default_tuning(step_mode=st.ST_STEP_PLAIN, **kw))
    _, d_s, n_s, s_s = gpu_render(sc, st.default_tuning(step_mode=st.ST_STEP_SEGMENT, **kw))
    print(f"\n[{sc.name}] plain steps {s_p['steps']} evals {s_p['field_evals']}; "
          f"segment steps {s_s['steps']} evals {s_s['field_evals']}", flush=True)
    return (d_p, n_p, s_p), (d_s, n_s, s_s)


@pytest.mark.parametrize("seed", [0, 3])
def test_segment_c1_full_image(seed):
    """First workload at its stated settings (128 steps, eps 1e-4)."""
    sc = sg.config1(seed)
    plain, seg = _pair(sc, max_steps=128, eps=1e-4)
    px, py = all_pixels(sc.camera)
    r = compare(sc, seg[0], seg[1], px, py)
    _report(f"c1 seed {seed} segment", r)
    assert seg[2]["unconverged"] == 0 and seg[2]["stalled"] == 0
    assert r["hits_oracle"] > 1000 and r["fail"] == 0, r
    assert_masks_agree(sc, seg[0], plain[0])
    assert seg[2]["steps"] < plain[2]["steps"]


@pytest.mark.parametrize("tile", [8, 32])
def test_segment_c2_full_image(tile):
    sc = sg.config2(0, 256, 256)
    plain, seg = _pair(sc, tile=tile)
    px, py = all_pixels(sc.camera)
    r = compare(sc, seg[0], seg[1], px, py)
    _report(f"c2 tile {tile} segment", r)
    assert seg[2]["stalled"] == 0 and seg[2]["unconverged"] == 0
    assert r["fail"] == 0, r
    assert_masks_agree(sc, seg[0], plain[0])
    assert seg[2]["steps"] < plain[2]["steps"]


@pytest.mark.timeout(600)
def test_segment_c3_stratified():
    """4096 primitives at 1920x1080: every GPU hit and its neighbours plus a
    seeded 16,384-pixel subset against the oracle; at least 2,000 hit rays."""
    sc = sg.config3(0)
    plain, seg = _pair(sc, tile=16, max_new=6, sub_depth=0.25)
    px, py = stratified_pixels(sc.camera, [seg[0], plain[0]], 16384, 5)
    r = compare(sc, seg[0], seg[1], px, py)
    _report("c3 segment stratified", r)
    assert seg[2]["stalled"] == 0 and seg[2]["unconverged"] == 0
    assert r["hits_compared"] >= 2000 and r["fail"] == 0, r
    assert seg[2]["steps"] <= plain[2]["steps"]
