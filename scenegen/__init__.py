"""Seeded synthetic blobtree scenes and cameras.

This module only draws random inputs: primitive parameters, tree shapes,
operator kinds and blend radii, and the pinhole camera.  It holds none of the
rendering method's arithmetic (no ranges of interest, no volumes of interest,
no operator formulas); both the GPU library and the CPU oracle consume the
arrays it returns.

Scene arrays (one row per blobtree node, any node order, ``root`` given):

* ``kind``  int32[N]   node kind, codes below
* ``left``, ``right`` int32[N]  child indices, -1 for primitives
* ``params`` float32[N, 16]  per-kind parameters:

  - SPHERE  : c(3), r
  - BOX     : c(3), half extents h(3), unit quaternion (w, x, y, z); the box
              axes are the columns of the quaternion's rotation matrix
  - CAPSULE : segment end a(3), segment end b(3), r
  - TORUS   : c(3), major radius R, minor radius r, unit quaternion (w, x, y, z);
              the ring lies in the local x-z plane around the local y axis
  - CYLINDER: c(3), radius, half height, unit quaternion; capped, its axis is
              the local y axis
  - CONE    : c(3), bottom radius, half height, unit quaternion, top radius;
              capped, its axis is the local y axis, the bottom disk at -h
  - UNION / INTER / DIFF (sharp CSG): no parameters
  - SUNION / SINTER / SDIFF (compact smooth CSG): k, d_o (d_o <= 0 asks the
    consumer to derive d_o from k)

All parameters are rounded to float32 here so that every consumer sees the
same numbers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SPHERE, BOX, CAPSULE, TORUS, CYLINDER, CONE = 0, 1, 2, 3, 4, 5
UNION, INTER, DIFF = 16, 17, 18
SUNION, SINTER, SDIFF = 19, 20, 21

# the primitive types of the configured workloads
PRIMITIVE_KINDS = (SPHERE, BOX, CAPSULE)
# every primitive type the library takes
EXTENDED_KINDS = (SPHERE, BOX, CAPSULE, TORUS, CYLINDER, CONE)
OPERATOR_KINDS = (UNION, INTER, DIFF, SUNION, SINTER, SDIFF)


@dataclass
class Camera:
    eye: tuple = (0.0, 0.0, 4.0)
    target: tuple = (0.0, 0.0, 0.0)
    up: tuple = (0.0, 1.0, 0.0)
    vfov_deg: float = 45.0
    width: int = 256
    height: int = 256


@dataclass
class Scene:
    name: str
    kind: np.ndarray
    left: np.ndarray
    right: np.ndarray
    params: np.ndarray
    root: int
    camera: Camera
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.kind.shape[0])

    @property
    def n_prims(self) -> int:
        return int(np.isin(self.kind, PRIMITIVE_KINDS).sum())


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _unit_quaternion(rng) -> np.ndarray:
    # uniformly distributed rotation (Shoemake's subgroup algorithm)
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([w, x, y, z])


def _unit_vector(rng) -> np.ndarray:
    while True:
        v = rng.normal(size=3)
        n = np.linalg.norm(v)
        if n > 1e-9:
            return v / n


class _Builder:
    def __init__(self):
        self.kind, self.left, self.right, self.params = [], [], [], []

    def add(self, kind, left=-1, right=-1, p=()):
        row = np.zeros(16, dtype=np.float64)
        row[: len(p)] = p
        self.kind.append(kind)
        self.left.append(left)
        self.right.append(right)
        self.params.append(row)
        return len(self.kind) - 1

    def finish(self, name, root, camera, meta) -> Scene:
        return Scene(
            name=name,
            kind=np.asarray(self.kind, dtype=np.int32),
            left=np.asarray(self.left, dtype=np.int32),
            right=np.asarray(self.right, dtype=np.int32),
            params=np.asarray(self.params, dtype=np.float32).reshape(-1, 16),
            root=int(root),
            camera=camera,
            meta=meta,
        )


def _primitive(rng, b: _Builder, centre, s, kinds=PRIMITIVE_KINDS):
    """One primitive of size s; the size law per type is fixed here."""
    t = kinds[int(rng.integers(len(kinds)))]
    c = np.asarray(centre, dtype=np.float64)
    if t == SPHERE:
        return b.add(SPHERE, p=(*c, s))
    if t == BOX:
        h = s * rng.uniform(0.5, 1.0, size=3)
        q = _unit_quaternion(rng)
        return b.add(BOX, p=(*c, *h, *q))
    if t == TORUS:
        R = s * rng.uniform(0.5, 1.0)
        r = R * rng.uniform(0.2, 0.5)
        q = _unit_quaternion(rng)
        return b.add(TORUS, p=(*c, R, r, *q))
    if t == CYLINDER:
        rad = s * rng.uniform(0.4, 1.0)
        h = s * rng.uniform(0.4, 1.0)
        q = _unit_quaternion(rng)
        return b.add(CYLINDER, p=(*c, rad, h, *q))
    if t == CONE:
        rb = s * rng.uniform(0.3, 1.0)
        rt = s * rng.uniform(0.0, 0.8)   # 0 to 0.8 s: pointed to nearly cylindrical
        h = s * rng.uniform(0.4, 1.0)
        q = _unit_quaternion(rng)
        return b.add(CONE, p=(*c, rb, h, *q, rt))
    u = _unit_vector(rng)
    a, e = c - 0.5 * s * u, c + 0.5 * s * u
    return b.add(CAPSULE, p=(*a, *e, 0.5 * s))


def _random_tree(rng, b: _Builder, leaves, max_depth, op_probs, k_range, ops=(SUNION, SINTER, SDIFF)):
    """Random binary tree over ``leaves`` (kept in order) with depth <= max_depth.

    A subtree of n leaves at depth l splits its leaves uniformly over the left
    sizes that still fit under the depth cap; each operator is drawn from
    ``ops`` with probabilities ``op_probs``."""
    if len(leaves) > 2 ** max_depth:
        raise ValueError("too many leaves for the depth cap")

    def build(lo, hi, depth):
        n = hi - lo
        if n == 1:
            return leaves[lo]
        cap = 2 ** (max_depth - depth - 1)
        nl_min, nl_max = max(1, n - cap), min(n - 1, cap)
        nl = int(rng.integers(nl_min, nl_max + 1))
        l = build(lo, lo + nl, depth + 1)
        r = build(lo + nl, hi, depth + 1)
        op = ops[int(rng.choice(len(ops), p=op_probs))]
        k = float(rng.uniform(*k_range))
        return b.add(op, l, r, (k, 0.0))

    return build(0, len(leaves), 0)


def config1(seed: int = 0, width: int = 256, height: int = 256) -> Scene:
    """16 spheres, centres U[-1,1]^3, radii U[0.1,0.3], balanced tree of compact
    smooth unions with blend radius 0.1; 256x256 camera at distance 4, 45 deg."""
    rng = _rng(seed)
    b = _Builder()
    level = []
    for _ in range(16):
        c = rng.uniform(-1.0, 1.0, size=3)
        r = rng.uniform(0.1, 0.3)
        level.append(b.add(SPHERE, p=(*c, r)))
    while len(level) > 1:
        level = [b.add(SUNION, level[i], level[i + 1], (0.1, 0.0)) for i in range(0, len(level), 2)]
    return b.finish("c1_16spheres", level[0], Camera(width=width, height=height),
                    {"config": 1, "seed": seed, "tile": 8})


def _mixed_scene(name, seed, n_prims, size_range, max_depth, width, height, tile,
                 centres=None, config=None, kinds=PRIMITIVE_KINDS, ops=(SUNION, SINTER, SDIFF),
                 op_probs=(0.6, 0.2, 0.2)):
    rng = _rng(seed)
    b = _Builder()
    if centres is None:
        centres = rng.uniform(-1.0, 1.0, size=(n_prims, 3))
    leaves = []
    for i in range(n_prims):
        s = float(rng.uniform(*size_range))
        leaves.append(_primitive(rng, b, centres[i], s, kinds=kinds))
    root = _random_tree(rng, b, leaves, max_depth, op_probs, (0.02, 0.15), ops=ops)
    return b.finish(name, root, Camera(width=width, height=height),
                    {"config": config, "seed": seed, "tile": tile, "max_depth": max_depth})


def config2(seed: int = 0, width: int = 1024, height: int = 1024, n_prims: int = 142,
            max_depth: int = 10) -> Scene:
    """142 spheres/boxes/capsules, sizes U[0.05,0.4], random tree of depth <= 10,
    compact smooth union/intersection/difference 60/20/20%, k U[0.02,0.15]; 1024^2."""
    return _mixed_scene(f"c2_{n_prims}prims", seed, n_prims, (0.05, 0.4), max_depth,
                        width, height, 16, config=2)


def config2_extended(seed: int = 0, width: int = 256, height: int = 256, n_prims: int = 142,
                     max_depth: int = 10) -> Scene:
    """The second workload's laws with every primitive type the library takes
    (sphere, box, capsule, torus, capped cylinder drawn uniformly): torus
    major radius s U[0.5,1] and minor radius R U[0.2,0.5], cylinder radius and
    half height s U[0.4,1], uniformly random orientations."""
    return _mixed_scene(f"c2x_{n_prims}prims", seed, n_prims, (0.05, 0.4), max_depth,
                        width, height, 16, config=2, kinds=EXTENDED_KINDS)


def config2_sharp(seed: int = 0, width: int = 256, height: int = 256, n_prims: int = 142,
                  max_depth: int = 10) -> Scene:
    """The second workload's primitives and tree shape with sharp operators
    beside the compact ones: union, intersection, difference sharp
    35/10/10%, compact 25/10/10% (creases where a sharp operator meets)."""
    return _mixed_scene(f"c2s_{n_prims}prims", seed, n_prims, (0.05, 0.4), max_depth, width, height, 16,
                        config=2, ops=(UNION, INTER, DIFF, SUNION, SINTER, SDIFF),
                        op_probs=(0.35, 0.1, 0.1, 0.25, 0.1, 0.1))


def gaussian_mixture_centres(rng, n, n_clusters=32, sigma=0.15):
    means = rng.uniform(-1.0, 1.0, size=(n_clusters, 3))
    comp = rng.integers(n_clusters, size=n)
    return means[comp] + sigma * rng.normal(size=(n, 3))


def config3(seed: int = 0, width: int = 1920, height: int = 1080, n_prims: int = 4096,
            max_depth: int = 16) -> Scene:
    """4096 primitives with the config-2 type and operator laws, sizes
    U[0.01,0.1], centres from a 32-cluster Gaussian mixture (sigma 0.15),
    random tree of depth <= 16; 1920x1080."""
    rng = _rng(seed + 0x5EED)
    centres = gaussian_mixture_centres(rng, n_prims)
    return _mixed_scene(f"c3_{n_prims}prims", seed, n_prims, (0.01, 0.1), max_depth,
                        width, height, 16, centres=centres, config=3)


C4_RESOLUTIONS = ((256, 256), (512, 512), (1024, 1024), (1920, 1080))


def config4_scene(i: int) -> Scene:
    """Scene i of the 64-scene batch: P log-uniform in [32, 8192], config-3
    generator, depth cap max(10, ceil(log2 P)+4), random resolution."""
    rng = _rng(1000 + i)
    p = int(round(math.exp(rng.uniform(math.log(32), math.log(8192)))))
    w, h = C4_RESOLUTIONS[int(rng.integers(len(C4_RESOLUTIONS)))]
    depth = max(10, math.ceil(math.log2(p)) + 4)
    sc = config3(seed=1000 + i, width=w, height=h, n_prims=p, max_depth=depth)
    sc.name = f"c4_{i:02d}_{p}prims_{w}x{h}"
    sc.meta["config"] = 4
    return sc


def config4(n_scenes: int = 64):
    return [config4_scene(i) for i in range(n_scenes)]


def config5(seed: int = 7777, width: int = 3840, height: int = 2160, n_prims: int = 16384,
            max_depth: int = 24) -> Scene:
    """Learned-step evaluation scene: 16384 primitives with the config-2 laws,
    depth cap 24, 3840x2160."""
    sc = _mixed_scene(f"c5_{n_prims}prims", seed, n_prims, (0.05, 0.4), max_depth,
                      width, height, 16, config=5)
    return sc


def single_primitive(kind: int, seed: int = 0, width: int = 64, height: int = 64) -> Scene:
    """One primitive near the origin (analytic-hit test scenes)."""
    rng = _rng(seed)
    b = _Builder()
    c = rng.uniform(-0.3, 0.3, size=3)
    root = _primitive(rng, b, c, float(rng.uniform(0.3, 0.8)), kinds=(kind,))
    return b.finish(f"single_{kind}", root, Camera(width=width, height=height, vfov_deg=25.0),
                    {"config": 0, "seed": seed, "tile": 8})


def random_small_tree(seed: int, n_leaves: int, ops=(SUNION, SINTER, SDIFF, UNION, INTER, DIFF),
                      size_range=(0.2, 0.6), spread=0.8, kinds=PRIMITIVE_KINDS,
                      k_range=(0.05, 0.3), width: int = 32, height: int = 32) -> Scene:
    """Small random trees (any shape, any operator mix) for exhaustive tests."""
    rng = _rng(seed)
    b = _Builder()
    leaves = [_primitive(rng, b, rng.uniform(-spread, spread, size=3),
                         float(rng.uniform(*size_range)), kinds=kinds) for _ in range(n_leaves)]

    def build(lo, hi):
        n = hi - lo
        if n == 1:
            return leaves[lo]
        nl = int(rng.integers(1, n))
        l, r = build(lo, lo + nl), build(lo + nl, hi)
        op = ops[int(rng.integers(len(ops)))]
        return b.add(op, l, r, (float(rng.uniform(*k_range)), 0.0))

    root = build(0, n_leaves)
    return b.finish(f"small_{seed}_{n_leaves}", root, Camera(width=width, height=height),
                    {"config": 0, "seed": seed, "tile": 8})


def tree_from_shape(shape, ops, seed: int = 0, kinds=(SPHERE,), k: float = 0.15,
                    spread: float = 0.6, size_range=(0.2, 0.5)) -> Scene:
    """Tree with a given nested-tuple shape, e.g. ((0, 0), 0) for a left comb of
    three leaves; ``ops`` lists operator kinds in post-order of the internal
    nodes."""
    rng = _rng(seed)
    b = _Builder()
    op_iter = iter(ops)

    def build(s):
        if not isinstance(s, tuple):
            c = rng.uniform(-spread, spread, size=3)
            return _primitive(rng, b, c, float(rng.uniform(*size_range)), kinds=kinds)
        l = build(s[0])
        r = build(s[1])
        return b.add(next(op_iter), l, r, (k, 0.0))

    root = build(shape)
    return b.finish("shaped", root, Camera(width=32, height=32), {"config": 0, "seed": seed})


def by_config(cfg: int, seed: int | None = None, **kw) -> Scene:
    fn = {1: config1, 2: config2, 3: config3, 5: config5}[cfg]
    if seed is None:
        return fn(**kw)
    return fn(seed=seed, **kw)
