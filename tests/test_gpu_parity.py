"""GPU parity of the HIP path against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_util import all_pixels, compare, gpu_render, sample_pixels, stratified_pixels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09673_amd import st
    st.lib()   # fails loudly without the built library


def _report(name, r):
    print(f"\n[{name}] " + " ".join(f"{k}={v}" for k, v in r.items() if k != "fail_idx"), flush=True)


# ---------------------------------------------------------------------------
# field evaluation

@pytest.mark.parametrize("make", [lambda: sg.config1(0), lambda: sg.config2(0), lambda: sg.random_small_tree(14, 9)],
                         ids=["c1", "c2", "small"])
def test_full_tree_field_matches_oracle(make):
    """All primitives active: the pruned view is the whole tree and f_A = f."""
    from paper_2304_09673_amd import st
    sc = make()
    s = st.Scene(sc)
    osc = oracle.OracleScene(sc)
    pts = np.random.default_rng(0).uniform(-1.3, 1.3, size=(4096, 3)).astype(np.float32)
    f, g, used, view = s.debug_eval(pts, None, grad=True)
    fo, go = osc.eval(pts.astype(np.float64), grad=True)
    f, g = f.cpu().numpy(), g.cpu().numpy()
    assert used == 1
    assert len(view) == sc.n_nodes
    err = np.abs(f - fo)
    assert err.max() < 2e-5 * (1 + np.abs(fo).max()), err.max()
    # gradients away from kinks
    ok = np.linalg.norm(g - go, axis=1) < 1e-3
    assert ok.mean() > 0.99


@pytest.mark.parametrize("make", [lambda: sg.config2(1), lambda: sg.config2(2), lambda: sg.random_small_tree(21, 12)],
                         ids=["c2s1", "c2s2", "small"])
def test_pruned_field_sign_equivalence(make):
    """Local equivalence (Section 3): with A the primitives whose volume of
    interest contains p, sign f_A(p) = sign f(p); the device view equals the
    host view of the same set."""
    from paper_2304_09673_amd import st
    sc = make()
    s = st.Scene(sc)
    osc = oracle.OracleScene(sc)
    prims = osc.prim_ids()
    rng = np.random.default_rng(1)
    n_checked = 0
    for _ in range(150):
        p = rng.uniform(-1.2, 1.2, size=3)
        act = [int(i) for i in prims if osc.in_voi(i, p)]
        if not act:
            continue
        f, _, used, view = s.debug_eval(p[None].astype(np.float32), act)
        host_view, _ = st.prune_tree(sc.kind, sc.left, sc.right, sc.params, sc.root, act)
        assert list(view) == list(host_view)
        fo = osc.eval(p[None])[0]
        fa = float(f.cpu().numpy()[0])
        if abs(fo) > 1e-4:
            assert (fa > 0) == (fo > 0), (p, act, fa, fo)
            n_checked += 1
    assert n_checked > 20


# ---------------------------------------------------------------------------
# A-buffer

@pytest.mark.parametrize("cfg,tile", [(1, 8), (2, 16), (2, 8), (2, 32)])
def test_abuffer_covers_every_ray_interval(cfg, tile):
    """Tile lists are a superset of the brute-force per-ray intervals: every
    primitive whose volume of interest meets a pixel-centre ray of the tile is
    listed with [z_in, z_out] covering that ray's interval; lists are sorted
    by (z_in, primitive)."""
    from paper_2304_09673_amd import st
    sc = sg.config1(0, 128, 128) if cfg == 1 else sg.config2(0, 96, 80)
    s = st.Scene(sc)
    s.build_abuffer(sc.camera, st.default_tuning(tile=tile, keep_all_entries=1))
    off, node, zin, zout = s.debug_abuffer()
    osc = oracle.OracleScene(sc)
    cam = sc.camera
    px, py = sample_pixels(cam, 600, 5)
    prims = osc.prim_ids()
    z = osc.voi_intervals(cam, px + 0.5, py + 0.5, prims)
    tiles_x = (cam.width + tile - 1) // tile
    for r in range(px.shape[0]):
        t = (py[r] // tile) * tiles_x + px[r] // tile
        seg = slice(off[t], off[t + 1])
        lst = {int(a): (float(b), float(c)) for a, b, c in zip(node[seg], zin[seg], zout[seg])}
        for q, i in enumerate(prims):
            z0, z1 = z[r, q]
            if np.isnan(z0):
                continue
            assert int(i) in lst, (r, i)
            a, b = lst[int(i)]
            assert a <= z0 + 1e-5 and b >= z1 - 1e-5, (a, b, z0, z1)
    # sorted by (z_in, primitive) per tile
    for t in range(off.shape[0] - 1):
        seg = slice(off[t], off[t + 1])
        keys = list(zip(zin[seg].tolist(), node[seg].tolist()))
        assert keys == sorted(keys)


def _tile_alive(sc, members):
    """Primitives of a tile's list that survive the dead-primitive rule for
    the whole list, written on the caller tree: a primitive is dropped when an
    ancestor on its path discards a lone operand from that side (an
    intersection, or a difference reached from the right) and no listed
    primitive is in the other operand; repeated until nothing drops."""
    parent, leaves = {}, {}

    def collect(v):
        if sc.kind[v] < 16:
            leaves[v] = frozenset([v])
        else:
            l, r = int(sc.left[v]), int(sc.right[v])
            parent[l], parent[r] = (v, 0), (v, 1)
            collect(l)
            collect(r)
            leaves[v] = leaves[l] | leaves[r]

    collect(int(sc.root))
    inter = {sg.INTER, sg.SINTER}
    diff = {sg.DIFF, sg.SDIFF}
    cur = set(members)
    while True:
        keep = set()
        for x in cur:
            v, alive = x, True
            while v in parent and alive:
                pv, side = parent[v]
                k = int(sc.kind[pv])
                kills = k in inter or (k in diff and side == 1)
                other = int(sc.right[pv]) if side == 0 else int(sc.left[pv])
                if kills and leaves[other].isdisjoint(cur):
                    alive = False
                v = pv
            if alive:
                keep.add(x)
        if keep == cur:
            return cur
        cur = keep


@pytest.mark.parametrize("which", ["c2", "c3small"])
def test_abuffer_pruning_keeps_the_tile_alive_set(which):
    """Tile-level pruning: each tile keeps exactly the entries of the
    primitives that survive the dead-primitive rule for the tile's whole
    binned list, with their depths, in (z_in, primitive) order; bit-exact
    against the rule evaluated on the host from the unpruned lists.  The
    candidates dropped before the per-ray test (dead for the tile's whole
    candidate set, or outside the screen rectangle of the other side of one
    of their killing ancestors) change nothing in the result."""
    from paper_2304_09673_amd import st
    sc = sg.config2(3, 160, 120) if which == "c2" else sg.config3(0, 192, 108, n_prims=512, max_depth=12)
    s = st.Scene(sc)
    s.build_abuffer(sc.camera, st.default_tuning(tile=16, keep_all_entries=1))
    off0, node0, zin0, zout0 = s.debug_abuffer()
    st0 = s.trace()[2]
    assert st0["abuffer_tested"] == st0["abuffer_candidates"]
    s.build_abuffer(sc.camera, st.default_tuning(tile=16))
    off1, node1, zin1, zout1 = s.debug_abuffer()
    st1 = s.trace()[2]
    assert st1["abuffer_candidates"] <= st0["abuffer_candidates"]
    assert st1["abuffer_entries"] <= st1["abuffer_binned"] <= st1["abuffer_tested"] <= st1["abuffer_candidates"]
    assert st1["abuffer_entries"] == int(off1[-1])
    assert off0.shape == off1.shape
    dropped = 0
    for t in range(off0.shape[0] - 1):
        a = slice(off0[t], off0[t + 1])
        full = {int(x): (zi, zo) for x, zi, zo in zip(node0[a], zin0[a].view(np.uint32), zout0[a].view(np.uint32))}
        alive = _tile_alive(sc, full.keys())
        b = slice(off1[t], off1[t + 1])
        kept = [int(x) for x in node1[b]]
        assert sorted(kept) == sorted(alive), t
        for x, zi, zo in zip(node1[b], zin1[b].view(np.uint32), zout1[b].view(np.uint32)):
            assert full[int(x)] == (zi, zo)
        keys = list(zip(zin1[b].tolist(), node1[b].tolist()))
        assert keys == sorted(keys)
        dropped += len(full) - len(kept)
    assert dropped > 0


def test_replayed_build_gives_the_same_image():
    """A second build with the same camera and tuning reruns the device work
    with the first build's sizes (no host synchronization): same A-buffer,
    bitwise the same image, same counters."""
    import torch
    from paper_2304_09673_amd import st
    sc = sg.config3(0, 320, 180, n_prims=1024, max_depth=12)
    s = st.Scene(sc)
    tune = st.default_tuning(tile=16, max_new=16)
    s.build_abuffer(sc.camera, tune)
    d0, n0, st0 = s.trace()
    a0 = s.debug_abuffer()
    d0, n0 = d0.cpu().numpy(), n0.cpu().numpy()
    for _ in range(2):
        s.build_abuffer(sc.camera, tune)
    d1, n1, st1 = s.trace()
    torch.cuda.synchronize()
    a1 = s.debug_abuffer()
    assert np.array_equal(d1.cpu().numpy(), d0) and np.array_equal(n1.cpu().numpy(), n0)
    for x, y in zip(a0, a1):
        assert np.array_equal(x, y)
    for k in ("hits", "field_evals", "subfrustums", "abuffer_entries", "abuffer_candidates"):
        assert st0[k] == st1[k], k


def test_abuffer_is_deterministic():
    from paper_2304_09673_amd import st
    sc = sg.config2(4, 128, 128)
    s = st.Scene(sc)
    s.build_abuffer(sc.camera)
    a = s.debug_abuffer()
    s.build_abuffer(sc.camera)
    b = s.debug_abuffer()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ---------------------------------------------------------------------------
# images

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c1_full_image_parity(seed):
    """16 spheres, compact smooth unions, 256x256, plain sphere tracing at the
    first workload's stated settings: at most 128 stepping evaluations per
    ray, eps 1e-4.  Every ray converges (none runs out of steps)."""
    from paper_2304_09673_amd import st
    sc = sg.config1(seed)
    s, depth, normal, stats = gpu_render(sc, st.default_tuning(max_steps=128, eps=1e-4))
    px, py = all_pixels(sc.camera)
    r = compare(sc, depth, normal, px, py)
    _report(f"c1 seed {seed} (128 steps)", r)
    print("stats", {k: stats[k] for k in ("rays", "hits", "unconverged", "field_evals", "steps", "subfrustums",
                                          "stalled")})
    assert stats["stalled"] == 0
    assert stats["unconverged"] == 0
    assert r["hits_oracle"] > 1000
    assert r["fail"] == 0, r


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_c2_parity_tiles(tile):
    """142 primitives, mixed compact operators, at 256x256 for every A-buffer
    tile size (the image must not depend on it)."""
    from paper_2304_09673_amd import st
    sc = sg.config2(0, 256, 256)
    s, depth, normal, stats = gpu_render(sc, st.default_tuning(tile=tile))
    px, py = all_pixels(sc.camera)
    r = compare(sc, depth, normal, px, py)
    _report(f"c2 tile {tile}", r)
    assert stats["stalled"] == 0
    assert r["fail"] == 0, r


def test_c2_full_resolution_sampled():
    sc = sg.config2(1)
    s, depth, normal, stats = gpu_render(sc)
    px, py = sample_pixels(sc.camera, 20000, 11)
    r = compare(sc, depth, normal, px, py)
    _report("c2 1024^2 sampled", r)
    assert r["hits_compared"] > 5000
    assert r["fail"] == 0, r


@pytest.mark.timeout(900)
def test_c3_stratified_parity():
    """4096 primitives at 1920x1080 in the launch configuration the benchmark
    times (the autotuner's choice): a seeded 65,536-pixel subset, every pixel
    the GPU hits and their neighbours, against the oracle.  The frame is
    mostly empty space (about 0.2% of pixels hit), so the hit pixels are taken
    whole: at least 2,000 compared hit rays."""
    from paper_2304_09673_amd import st
    sc = sg.config3(0)
    s = st.Scene(sc)
    tune, ms = s.autotune(sc.camera, reps=1)
    print(f"\n[c3] autotuned tile {tune.tile} max_new {tune.max_new} sub_depth {tune.sub_depth:.4g} ({ms:.3f} ms)",
          flush=True)
    depth, normal, stats = s.trace()
    depth, normal = depth.cpu().numpy(), normal.cpu().numpy()
    px, py = stratified_pixels(sc.camera, [depth], 65536, 12)
    print(f"[c3] comparing {px.shape[0]} pixels ({int(np.isfinite(depth).sum())} GPU hits)", flush=True)
    r = compare(sc, depth, normal, px, py)
    _report("c3 stratified", r)
    assert stats["stalled"] == 0 and stats["unconverged"] == 0
    assert r["hits_compared"] >= 2000, r
    assert r["fail"] == 0, r


def test_camera_facing_away_gives_an_empty_image():
    """A build with no candidate at all (every volume of interest behind the
    eye) still writes the dispatch order the trace reads: every pixel is a
    miss (+inf depth, zero normal), every ray is counted."""
    import torch
    from paper_2304_09673_amd import st
    sc = sg.config1(0, 96, 80)
    cam = sg.Camera(width=96, height=80, eye=(0.0, 0.0, 4.0), target=(0.0, 0.0, 8.0))
    s = st.Scene(sc)
    for tile in (8, 16, 32):
        s.build_abuffer(cam, st.default_tuning(tile=tile))
        depth = torch.full((cam.height, cam.width), -1.0, device="cuda")
        normal = torch.full((cam.height, cam.width, 3), -1.0, device="cuda")
        _, _, stats = s.trace(cam, depth, normal)
        torch.cuda.synchronize()
        assert stats["abuffer_candidates"] == 0
        assert stats["rays"] == cam.width * cam.height
        assert stats["hits"] == 0 and stats["stalled"] == 0
        assert torch.isinf(depth).all() and bool((depth > 0).all())
        assert bool((normal == 0).all())


@pytest.mark.parametrize("n_prims,max_active", [(142, 4), (1024, 16)])
def test_small_capacity_runs_the_wide_path_with_the_same_image(n_prims, max_active):
    """Tiles whose volumes of interest overlap more than max_active run on the
    wide-capacity path (never a failure): the image is bitwise that of the
    default capacity, and matches the oracle.  The second workload's laws at
    256x256; with 142 primitives the kept overlap reaches 8, with 1024 it
    passes 16."""
    from paper_2304_09673_amd import st
    sc = sg.config2(0, 256, 256, n_prims=n_prims)
    _, d0, n0, s0 = gpu_render(sc, st.default_tuning())
    _, d1, n1, s1 = gpu_render(sc, st.default_tuning(max_active=max_active))
    print(f"\n[capacity {max_active}] wide tiles {s1['wide_tiles']} (default {s0['wide_tiles']}), "
          f"largest overlap {s1['max_overlap']}", flush=True)
    assert s0["wide_tiles"] == 0
    assert s1["wide_tiles"] > 0
    assert s1["max_overlap"] > max_active
    np.testing.assert_array_equal(d1, d0)
    np.testing.assert_array_equal(n1, n0)
    px, py = all_pixels(sc.camera)
    r = compare(sc, d1, n1, px[::2], py[::2])
    assert r["fail"] == 0, r


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_autotuned_tuning_passes_parity(which):
    """st_autotune picks tile size and fetch parameters by timing; whatever it
    picks, the image meets the parity rules."""
    from paper_2304_09673_amd import st
    sc = sg.config1(1, 192, 192) if which == "c1" else sg.config2(2, 256, 256)
    s = st.Scene(sc)
    tune, ms = s.autotune(sc.camera, reps=1)
    assert tune.tile in (8, 16, 32) and ms > 0
    depth, normal, stats = s.trace()
    px, py = all_pixels(sc.camera)
    r = compare(sc, depth.cpu().numpy(), normal.cpu().numpy(), px, py)
    _report(f"{which} autotuned tile {tune.tile} max_new {tune.max_new} sub {tune.sub_depth:.3g}", r)
    assert stats["stalled"] == 0
    assert r["fail"] == 0, r


def test_trace_rejects_stale_camera():
    from paper_2304_09673_amd import st
    sc = sg.config1(0, 64, 64)
    s = st.Scene(sc)
    s.build_abuffer(sc.camera)
    other = sg.Camera(width=64, height=64, eye=(0.0, 0.5, 4.0))
    with pytest.raises(st.StError) as e:
        s.trace(other)
    assert e.value.code == st.ST_E_STALE


@pytest.mark.parametrize("which", ["c3", "c5"])
def test_device_view_equals_host_view_large_sets(which):
    """Random active sets of 2 to 1000 primitives (scattered and contiguous in
    post-order): the device view (dead-primitive filter, both ordering paths,
    the bottom-up pass) equals the host view of the same set."""
    from paper_2304_09673_amd import st
    sc = sg.config3() if which == "c3" else sg.config5(width=64, height=64)
    s = st.Scene(sc)
    prims = np.nonzero(np.isin(sc.kind, sg.PRIMITIVE_KINDS))[0]
    rng = np.random.default_rng(5 if which == "c3" else 6)
    n_used = 0
    for size in (2, 3, 5, 30, 63, 64, 65, 129, 200, 511, 700, 1000):
        for contiguous in (False, True):
            if contiguous:
                # primitives generated together: often one region of the tree
                start = int(rng.integers(0, len(prims) - size))
                act = prims[start:start + size]
            else:
                act = rng.choice(prims, size=size, replace=False)
            act = [int(a) for a in act]
            pt = np.zeros((1, 3), dtype=np.float32)
            _, _, used, view = s.debug_eval(pt, act)
            host_view, _ = st.prune_tree(sc.kind, sc.left, sc.right, sc.params, sc.root, act)
            assert list(view) == list(host_view), (which, size, contiguous)
            n_used += int(used)
    if which == "c3":
        # (the 16384-primitive tree is intersection-heavy: random sets of its
        # primitives almost never reach the root, which the equality above
        # covers as well)
        assert n_used > 0


def test_block_clock_counters():
    """Per-block shader clock counters: the longest block is at least the mean,
    and the longest block, converted at a 2.5 GHz clock (above the chip's
    highest), does not exceed the launch's duration measured with HIP events."""
    import torch
    from paper_2304_09673_amd import st
    sc = sg.config2(0, 256, 256)
    s = st.Scene(sc)
    s.build_abuffer(sc.camera, st.default_tuning(tile=16))
    s.trace()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    _, _, stats = s.trace()
    b.record()
    torch.cuda.synchronize()
    blocks = (256 // 8) * (256 // 8)
    mx, mean = stats["block_cycles_max"], stats["block_cycles_sum"] / blocks
    assert 0 < mean <= mx, stats
    assert mx / 2.5e9 * 1e3 <= a.elapsed_time(b) + 0.01, (mx, a.elapsed_time(b))
