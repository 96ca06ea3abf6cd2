"""CPU-side checks of the C ABI library: it loads without a GPU, exports every
function include/st.h declares, and its host logic (flatten validation, the
pruned tree view) follows the paper's rules."""
import ast
import ctypes as C
import itertools
import re
from pathlib import Path

import numpy as np
import pytest

import scenegen as sg
from paper_2304_09673_amd import st

ROOT = Path(__file__).resolve().parents[1]


def _declared():
    text = (ROOT / "include" / "st.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(st_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 11
    lib = st.lib()
    for n in names:
        assert hasattr(lib, n), n
        assert n in st.EXPORTS, n
    assert set(st.EXPORTS) == set(names)


def test_binding_loads_one_hip_runtime():
    """Loading the library through the binding in a fresh process maps a
    single HIP runtime (torch's): the library binds to the runtime torch
    already loaded instead of bringing a second one."""
    import subprocess
    import sys
    code = ("from paper_2304_09673_amd import st; st.lib(); "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=str(Path(__file__).resolve().parents[1]), check=True).stdout
    paths = ast.literal_eval(out.strip().splitlines()[-1])
    assert len(paths) == 1, paths


def test_status_strings_and_default_tuning():
    lib = st.lib()
    assert lib.st_status_str(0) == b"ok"
    assert lib.st_status_str(6) == b"stale A-buffer"
    t = st.default_tuning()
    # the paper's defaults (Implementation details): 8x8 tiles are the trace
    # granularity; d = 1/20 of scene depth, <= 6 new primitives per fetch
    assert abs(t.sub_depth - 0.05) < 1e-7 and t.max_new == 6
    assert t.eps == pytest.approx(1e-4) and t.max_steps == 1024
    assert abs(t.omega - 1.7) < 1e-6


# ---------------------------------------------------------------------------
# flatten validation (host only)

def _prune(sc, active):
    return st.prune_tree(sc.kind, sc.left, sc.right, sc.params, sc.root, active)


def test_flatten_rejects_malformed_trees():
    sc = sg.random_small_tree(1, 4)
    # cycle: a child points back to the root
    k, l, r, p = sc.kind.copy(), sc.left.copy(), sc.right.copy(), sc.params.copy()
    op = int(np.nonzero(k >= 16)[0][0])
    l[op] = sc.root
    with pytest.raises(st.StError) as e:
        st.prune_tree(k, l, r, p, sc.root, [])
    assert e.value.code == st.ST_E_TREE
    # unknown kind
    k = sc.kind.copy()
    k[0] = 7
    with pytest.raises(st.StError) as e:
        st.prune_tree(k, sc.left, sc.right, sc.params, sc.root, [])
    assert e.value.code == st.ST_E_TREE
    # unreachable node (extra primitive)
    k = np.append(sc.kind, sg.SPHERE).astype(np.int32)
    l = np.append(sc.left, -1).astype(np.int32)
    r = np.append(sc.right, -1).astype(np.int32)
    p = np.vstack([sc.params, sc.params[:1]])
    with pytest.raises(st.StError) as e:
        st.prune_tree(k, l, r, p, sc.root, [])
    assert e.value.code == st.ST_E_TREE


@pytest.mark.parametrize("field,value", [("radius", 0.0), ("radius", float("nan")), ("k", -0.1), ("k", float("inf"))])
def test_flatten_rejects_bad_parameters(field, value):
    sc = sg.tree_from_shape((0, 0), [sg.SUNION])
    p = sc.params.copy()
    if field == "radius":
        p[sc.left[sc.root], 3] = value
    else:
        p[sc.root, 0] = value
    with pytest.raises(st.StError) as e:
        st.prune_tree(sc.kind, sc.left, sc.right, p, sc.root, [])
    assert e.value.code == st.ST_E_INVALID


@pytest.mark.parametrize("kind", [sg.TORUS, sg.CYLINDER])
@pytest.mark.parametrize("col,value", [(3, 0.0), (4, -0.2), (4, float("nan")), ("quat", 0.0)])
def test_flatten_rejects_bad_torus_and_cylinder_parameters(kind, col, value):
    """Radii (torus R and r; cylinder radius and half height) must be > 0 and
    finite, the quaternion non-zero; a valid one flattens."""
    sc = sg.tree_from_shape((0, 0), [sg.SUNION], kinds=(kind,))
    st.prune_tree(sc.kind, sc.left, sc.right, sc.params, sc.root, [])
    p = sc.params.copy()
    leaf = sc.left[sc.root]
    if col == "quat":
        p[leaf, 5:9] = 0.0
    else:
        p[leaf, col] = value
    with pytest.raises(st.StError) as e:
        st.prune_tree(sc.kind, sc.left, sc.right, p, sc.root, [])
    assert e.value.code == st.ST_E_INVALID


def test_flatten_rejects_too_deep_tree():
    # left comb of 33 leaves: depth 32 > 31
    shape = 0
    for _ in range(32):
        shape = (shape, 0)
    sc = sg.tree_from_shape(shape, [sg.UNION] * 32)
    with pytest.raises(st.StError) as e:
        _prune(sc, [])
    assert e.value.code == st.ST_E_TREE


# ---------------------------------------------------------------------------
# Pruned view semantics (Sections 7-9): expected view computed recursively
# from the paper's rules, independently of the library's LCA construction.
ABSENT, UNUSED = "absent", "unused"
IGNORE = {sg.UNION: 0, sg.SUNION: 0, sg.INTER: 3, sg.SINTER: 3, sg.DIFF: 2, sg.SDIFF: 2}


def _expected(sc, active):
    """Post-order list of the evaluated nodes and the view's Lipschitz bound.

    A subtree without active primitive is absent.  An operator whose
    operand usage bits b = (left used << 1) | right used satisfy
    (~b & ignoreMod) == 0 takes op_type b, else 0 (Section 9):
    3 evaluates the operator, 2 returns the left operand, 1 the right one,
    0 returns +inf (the branch is unused)."""
    act = set(int(a) for a in active)

    def lipf(v):
        if sc.kind[v] >= sg.SUNION:
            k = float(sc.params[v, 0])
            d = float(sc.params[v, 1]) if sc.params[v, 1] > 0 else 7 * k / 6
            return 1 + k / (6 * d - k)
        return 1.0

    def rec(v):
        if sc.kind[v] < 16:
            return ([v], 1.0) if v in act else ABSENT
        a, b = rec(sc.left[v]), rec(sc.right[v])
        if a == ABSENT and b == ABSENT:
            return ABSENT
        lu = 0 if a in (ABSENT, UNUSED) else 1
        ru = 0 if b in (ABSENT, UNUSED) else 1
        bits = (lu << 1) | ru
        im = IGNORE[int(sc.kind[v])]
        op = bits if ((~bits & im) & 3) == 0 else 0
        if op == 3:
            return (a[0] + b[0] + [v], max(a[1], b[1]) * lipf(v))
        if op == 2:
            return a
        if op == 1:
            return b
        return UNUSED

    r = rec(sc.root)
    if r in (ABSENT, UNUSED):
        return [], 0.0
    return r[0], r[1]


def _shapes(n):
    if n == 1:
        yield 0
        return
    for k in range(1, n):
        for a in _shapes(k):
            for b in _shapes(n - k):
                yield (a, b)


OPS = [sg.UNION, sg.INTER, sg.DIFF, sg.SUNION, sg.SINTER, sg.SDIFF]


@pytest.mark.parametrize("n_leaves", [1, 2, 3, 4, 5, 6])
def test_prune_exhaustive_small_trees(n_leaves):
    """Every tree shape with n leaves, several operator assignments, every
    active subset."""
    rng = np.random.default_rng(n_leaves)
    cases = 0
    for shape in _shapes(n_leaves):
        n_ops = n_leaves - 1
        assigns = [[op] * n_ops for op in OPS] if n_ops else [[]]
        assigns += [list(rng.choice(OPS, n_ops)) for _ in range(4)] if n_ops else []
        for ops in assigns:
            sc = sg.tree_from_shape(shape, ops, seed=cases, k=float(rng.uniform(0.05, 0.3)))
            prims = np.nonzero(sc.kind < 16)[0]
            for mask in range(1 << n_leaves):
                active = [int(prims[i]) for i in range(n_leaves) if mask >> i & 1]
                got, lip = _prune(sc, active)
                exp, elip = _expected(sc, active)
                assert list(got) == exp, (shape, ops, active)
                assert lip == pytest.approx(elip, rel=1e-6)
                cases += 1
    assert cases > 0


@pytest.mark.parametrize("seed", range(8))
def test_prune_random_larger_trees(seed):
    rng = np.random.default_rng(100 + seed)
    for rep in range(40):
        n = int(rng.integers(7, 40))
        sc = sg.random_small_tree(seed * 1000 + rep, n, ops=tuple(OPS))
        prims = np.nonzero(sc.kind < 16)[0]
        for _ in range(10):
            active = [int(p) for p in prims if rng.random() < rng.uniform(0.1, 0.9)]
            got, lip = _prune(sc, active)
            exp, elip = _expected(sc, active)
            assert list(got) == exp
            assert lip == pytest.approx(elip, rel=1e-6)


# ---------------------------------------------------------------------------
# Algorithm 1 (sparse bottom-up traversal with direct evaluation), parent and
# fast ancestor pointers: the expression it evaluates must be the pruned view
# of the rules above, for every shape, operator mix and active subset.

def _sparse(sc, active, variant):
    from paper_2304_09673_amd import st
    return st.sparse_traversal(sc.kind, sc.left, sc.right, sc.params, sc.root, active, variant)


@pytest.mark.parametrize("n_leaves", [1, 2, 3, 4, 5, 6])
def test_sparse_traversal_exhaustive_small_trees(n_leaves):
    from paper_2304_09673_amd import st
    rng = np.random.default_rng(50 + n_leaves)
    cases = 0
    for shape in _shapes(n_leaves):
        n_ops = n_leaves - 1
        assigns = [[op] * n_ops for op in OPS] if n_ops else [[]]
        assigns += [list(rng.choice(OPS, n_ops)) for _ in range(4)] if n_ops else []
        for ops in assigns:
            sc = sg.tree_from_shape(shape, ops, seed=cases, k=float(rng.uniform(0.05, 0.3)))
            prims = np.nonzero(sc.kind < 16)[0]
            for mask in range(1 << n_leaves):
                active = [int(prims[i]) for i in range(n_leaves) if mask >> i & 1]
                exp, elip = _expected(sc, active)
                vis = {}
                for variant in (st.ST_ABLATION_PARENT_PTR, st.ST_ABLATION_FAST_PTR):
                    got, lip, vis[variant] = _sparse(sc, active, variant)
                    assert list(got) == exp, (shape, ops, active, variant)
                    assert lip == pytest.approx(elip, rel=1e-6)
                assert vis[st.ST_ABLATION_FAST_PTR] <= vis[st.ST_ABLATION_PARENT_PTR]
                cases += 1
    assert cases > 0


@pytest.mark.parametrize("seed", range(6))
def test_sparse_traversal_random_larger_trees(seed):
    """Random trees of 7 to 60 leaves (deep and lopsided shapes), random
    active subsets: both pointer variants give the pruned view."""
    from paper_2304_09673_amd import st
    rng = np.random.default_rng(300 + seed)
    for rep in range(40):
        n = int(rng.integers(7, 60))
        sc = sg.random_small_tree(seed * 1000 + rep, n, ops=tuple(OPS))
        prims = np.nonzero(sc.kind < 16)[0]
        for _ in range(10):
            active = [int(p) for p in prims if rng.random() < rng.uniform(0.05, 0.9)]
            exp, elip = _expected(sc, active)
            for variant in (st.ST_ABLATION_PARENT_PTR, st.ST_ABLATION_FAST_PTR):
                got, lip, _ = _sparse(sc, active, variant)
                assert list(got) == exp, (seed, rep, variant)
                assert lip == pytest.approx(elip, rel=1e-6)


def test_fast_pointers_skip_the_spine_of_a_left_comb():
    """A left comb of unions with only its deepest primitive active: parent
    pointers visit every spine operator, fast pointers jump to the root at
    once (the left-heavy case the paper introduces them for)."""
    from paper_2304_09673_amd import st
    n_leaves = 12
    shape = 0
    for _ in range(n_leaves - 1):
        shape = (shape, 0)
    sc = sg.tree_from_shape(shape, [sg.SUNION] * (n_leaves - 1))
    prims = np.nonzero(sc.kind < 16)[0]
    deepest = int(min(prims))
    for variant, want in ((st.ST_ABLATION_PARENT_PTR, n_leaves - 1), (st.ST_ABLATION_FAST_PTR, 1)):
        got, _, vis = _sparse(sc, [deepest], variant)
        assert list(got) == [deepest] and vis == want, (variant, vis)


def _kill_filter(sc, active):
    """The dead-primitive rule of the device view build, written on the tree:
    a primitive is dropped when some ancestor on its path discards a lone
    operand from that side (an intersection, or a difference reached from
    the right) and no active primitive is in the other operand; applied
    until nothing more drops."""
    parent = {}
    for v in range(len(sc.kind)):
        if sc.kind[v] >= 16:
            parent[int(sc.left[v])] = (v, 0)
            parent[int(sc.right[v])] = (v, 1)

    def leaves(v):
        return [v] if sc.kind[v] < 16 else leaves(int(sc.left[v])) + leaves(int(sc.right[v]))

    act = set(active)
    while True:
        keep = set()
        for x in act:
            v, alive = x, True
            while v in parent and alive:
                pv, side = parent[v]
                im = IGNORE[int(sc.kind[pv])]
                kills = (im & 1) if side == 0 else (im & 2)
                other = int(sc.right[pv]) if side == 0 else int(sc.left[pv])
                if kills and not act.intersection(leaves(other)):
                    alive = False
                v = pv
            if alive:
                keep.add(x)
        if keep == act:
            return sorted(act)
        act = keep


@pytest.mark.parametrize("seed", range(4))
def test_dead_primitive_filter_keeps_the_view(seed):
    """Dropping the primitives that the kill-chain rule finds dead, to a fixed
    point, gives the same view as the full active set (the view-build filter
    changes only the work, never the view)."""
    rng = np.random.default_rng(500 + seed)
    dropped = 0
    for rep in range(40):
        n = int(rng.integers(5, 30))
        sc = sg.random_small_tree(seed * 1000 + rep, n, ops=tuple(OPS))
        prims = np.nonzero(sc.kind < 16)[0]
        for _ in range(10):
            active = sorted(int(p) for p in prims if rng.random() < rng.uniform(0.1, 0.9))
            kept = _kill_filter(sc, active)
            dropped += len(active) - len(kept)
            assert _expected(sc, kept) == _expected(sc, active)
    assert dropped > 0


def _cut_by_ancestors(sc, cand, hits):
    """The candidates left by the killing-ancestor cut, written on sets: a
    candidate goes when one of its killing ancestors (an intersection, or a
    difference reached from the right) has no hit in its other operand."""
    parent = {}
    for v in range(len(sc.kind)):
        if sc.kind[v] >= 16:
            parent[int(sc.left[v])] = (v, 0)
            parent[int(sc.right[v])] = (v, 1)

    def leaves(v):
        return [v] if sc.kind[v] < 16 else leaves(int(sc.left[v])) + leaves(int(sc.right[v]))

    h = set(hits)
    out = []
    for x in cand:
        v, ok = x, True
        while v in parent and ok:
            pv, side = parent[v]
            im = IGNORE[int(sc.kind[pv])]
            kills = (im & 1) if side == 0 else (im & 2)
            other = int(sc.right[pv]) if side == 0 else int(sc.left[pv])
            if kills and not h.intersection(leaves(other)):
                ok = False
            v = pv
        if ok:
            out.append(x)
    return out


@pytest.mark.parametrize("seed", range(4))
def test_candidate_cuts_keep_the_alive_set(seed):
    """The binning's three cuts leave a tile the primitives alive for its
    hits H, whatever superset C of H its candidates are: the killing-ancestor
    cut keeps every primitive alive for H; the rule on the remaining
    candidates keeps them too; and the rule on the hits left by both gives
    alive(H), as it does from any set between alive(H) and H."""
    rng = np.random.default_rng(700 + seed)
    cut = 0
    for rep in range(30):
        n = int(rng.integers(5, 30))
        sc = sg.random_small_tree(seed * 1000 + rep, n, ops=tuple(OPS))
        prims = [int(p) for p in np.nonzero(sc.kind < 16)[0]]
        for _ in range(8):
            cand = sorted(p for p in prims if rng.random() < rng.uniform(0.3, 1.0))
            hits = sorted(p for p in cand if rng.random() < rng.uniform(0.2, 1.0))
            alive_h = _kill_filter(sc, hits)
            c1 = _cut_by_ancestors(sc, cand, hits)
            assert set(alive_h) <= set(c1)
            c2 = _kill_filter(sc, c1)
            assert set(alive_h) <= set(c2)
            tested_hits = sorted(set(hits) & set(c2))
            assert _kill_filter(sc, tested_hits) == alive_h
            between = sorted(set(alive_h) | {x for x in hits if rng.random() < 0.5})
            assert _kill_filter(sc, between) == alive_h
            cut += len(cand) - len(c2)
    assert cut > 0


def test_prune_left_comb_union_only_keeps_active_operators():
    """Left comb of unions (Section 7 inset): with k active primitives the
    view holds those k primitives and k-1 operators, never the skipped ones."""
    shape = 0
    for _ in range(9):
        shape = (shape, 0)
    sc = sg.tree_from_shape(shape, [sg.SUNION] * 9)
    prims = list(np.nonzero(sc.kind < 16)[0])
    got, lip = _prune(sc, [prims[2], prims[7]])
    assert len(got) == 3
    assert lip == pytest.approx(7 / 6, rel=1e-6)


def test_prune_intersection_with_lone_operand_is_unused():
    """Section 9: an intersection with one active operand is ignored; a
    difference without its left operand too; with only its left operand it
    returns it."""
    sc = sg.tree_from_shape((0, 0), [sg.SINTER])
    a, b = sc.left[sc.root], sc.right[sc.root]
    assert len(_prune(sc, [a])[0]) == 0
    assert len(_prune(sc, [a, b])[0]) == 3
    sc = sg.tree_from_shape((0, 0), [sg.SDIFF])
    a, b = sc.left[sc.root], sc.right[sc.root]
    assert list(_prune(sc, [a])[0]) == [a]
    assert len(_prune(sc, [b])[0]) == 0


def test_golden_single_operator_views():
    """The per-operator behaviour the paper tabulates (ignoreMod codes and the
    reserved op types), for sharp and compact smooth operators of each class."""
    from pathlib import Path
    rows = []
    for line in (Path(__file__).parent / "golden" / "ignoremod_single_operator.txt").read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            parts = line.split()
            rows.append((parts[0], parts[1], parts[2:]))
    assert len(rows) == 12
    kinds = {"union": (sg.UNION, sg.SUNION), "intersection": (sg.INTER, sg.SINTER),
             "difference": (sg.DIFF, sg.SDIFF)}
    for cls, active, expect in rows:
        for k in kinds[cls]:
            kind = np.array([sg.SPHERE, sg.SPHERE, k], dtype=np.int32)
            left = np.array([-1, -1, 0], dtype=np.int32)
            right = np.array([-1, -1, 1], dtype=np.int32)
            params = np.zeros((3, 16), dtype=np.float32)
            params[0, :4] = [-0.2, 0, 0, 0.5]
            params[1, :4] = [0.2, 0, 0, 0.5]
            params[2, :2] = [0.1, 0.0]
            act = [] if active == "-" else [{"A": 0, "B": 1}[c] for c in active]
            view, _ = st.prune_tree(kind, left, right, params, 2, act)
            names = {0: "A", 1: "B", 2: "op"}
            got = [names[int(v)] for v in view] or ["-"]
            assert got == expect, (cls, k, active, got, expect)


def test_train_step_model_refuses_bad_arguments():
    """Argument checks of st_train_step_model come before any device work."""
    import ctypes as C
    L = st.lib()
    buf = (C.c_float * 16)()
    p = C.cast(buf, C.c_void_p)
    ok = dict(x=p, t=p, n=10, epochs=1, batch=4, lr=1e-3, over=4.0, w=p, norm=p)
    for bad in (dict(x=None), dict(t=None), dict(w=None), dict(norm=None), dict(n=0), dict(n=1 << 31),
                dict(epochs=0), dict(batch=0), dict(lr=0.0), dict(lr=float("nan")), dict(over=0.0)):
        a = {**ok, **bad}
        r = L.st_train_step_model(a["x"], a["t"], a["n"], a["epochs"], a["batch"], a["lr"], a["over"], 0,
                                  a["w"], a["norm"], None, None)
        assert r == st.ST_E_INVALID, bad


@pytest.mark.parametrize("col,value", [(3, -0.1), (9, -0.1), ("both", 0.0), (4, 0.0), (9, float("nan")), ("quat", 0.0)])
def test_flatten_rejects_bad_cone_parameters(col, value):
    """Cone radii must be >= 0 and not both 0, the half height > 0, every
    parameter finite, the quaternion non-zero; a valid one flattens."""
    sc = sg.tree_from_shape((0, 0), [sg.SUNION], kinds=(sg.CONE,))
    st.prune_tree(sc.kind, sc.left, sc.right, sc.params, sc.root, [])
    p = sc.params.copy()
    leaf = sc.left[sc.root]
    if col == "quat":
        p[leaf, 5:9] = 0.0
    elif col == "both":
        p[leaf, 3] = p[leaf, 9] = 0.0
    else:
        p[leaf, col] = value
    with pytest.raises(st.StError) as e:
        st.prune_tree(sc.kind, sc.left, sc.right, p, sc.root, [])
    assert e.value.code == st.ST_E_INVALID
