"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each pin uses a computation different from the oracle's own (ray/surface
intersections instead of root finding on a distance field, hand-derived
closed forms, brute force, invariants), so that a dropped term, a wrong sign
or a transposed operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg

K = 0.1


def _op_scene(kind, k=K, d_o=0.0):
    """Two-sphere tree whose root is operator `kind` (only the operator's own
    evaluation on given operand values is used)."""
    kind_a = np.array([sg.SPHERE, sg.SPHERE, kind], dtype=np.int32)
    left = np.array([-1, -1, 0], dtype=np.int32)
    right = np.array([-1, -1, 1], dtype=np.int32)
    p = np.zeros((3, 16), dtype=np.float32)
    p[0, :4] = (0, 0, 0, 0.5)
    p[1, :4] = (0.3, 0, 0, 0.5)
    p[2, :2] = (k, d_o)
    return oracle.OracleScene(kind=kind_a, left=left, right=right, params=p, root=2)


# ---------------------------------------------------------------------------
# Operators: closed forms derived by hand from eq. (smooth-union)..(smooth-diff),
# eq. (smooth_comp) and eq. (compact_smooth_union), with d_o = 7k/6, so that
# 6 d_o - k = 6k and b_r(x) = k max(1 - x/k, 0).

def test_sharp_csg_closed_forms():
    for kind, fn in ((sg.UNION, min), (sg.INTER, max), (sg.DIFF, lambda a, b: max(a, -b))):
        o = _op_scene(kind)
        rng = np.random.default_rng(0)
        for a, b in rng.uniform(-1, 1, size=(200, 2)):
            assert o.op(2, a, b) == fn(a, b)


def test_compact_union_closed_forms():
    o = _op_scene(sg.SUNION)
    k = np.float64(np.float32(K))
    assert o.d_o(2) == pytest.approx(7 * k / 6, rel=1e-15)
    # a = b = 0: x = -k/6, K = 7k/6, G = -K/6 = -7k/36
    assert o.op(2, 0.0, 0.0) == pytest.approx(-7 * k / 36, rel=1e-13)
    # on the iso-surface of the unmodified blend (a = b = k/6: g(k) = 0) the
    # blend radius is k and the compact operator returns g(k) = 0
    assert abs(o.op(2, k / 6, k / 6)) < 1e-15
    # operands far apart (|a-b| >= blend radius): plain min
    assert o.op(2, -0.5, 0.3) == -0.5
    # one operand outside R_o = (-inf, 7k/6]: sharp union
    assert o.op(2, 7 * k / 6 + 1e-9, 0.1) == 0.1
    # a = 0, b = k/2 by hand: x = -k/6 (1/2)^3, K = k - x,
    # G = -K/6 (1 - (k/2)/K)^3
    x = -k / 6 * 0.125
    Kb = k - x
    expect = -Kb / 6 * (1 - (k / 2) / Kb) ** 3
    assert o.op(2, 0.0, k / 2) == pytest.approx(expect, rel=1e-13)


def test_compact_intersection_and_difference_closed_forms():
    k = np.float64(np.float32(K))
    oi = _op_scene(sg.SINTER)
    # a = b = 0: x = k/6, K = min(k - k/6, k) = 5k/6, G = 0 + K/6 = 5k/36
    assert oi.op(2, 0.0, 0.0) == pytest.approx(5 * k / 36, rel=1e-13)
    # iso-surface of g_inter(k): a = b = -k/6 -> G = 0
    assert abs(oi.op(2, -k / 6, -k / 6)) < 1e-15
    # deep inside both: x < 0 so b_r > k, clamped to k: G = g_inter(a, b, k)
    a, b = -0.5, -0.45
    h = 1 - abs(a - b) / k
    assert oi.op(2, a, b) == pytest.approx(max(a, b) + k / 6 * h ** 3, rel=1e-13)
    od = _op_scene(sg.SDIFF)
    # a = 0, b = 0: x = max(0, -0) + k/6 = k/6, K = 5k/6, G = 5k/36
    assert od.op(2, 0.0, 0.0) == pytest.approx(5 * k / 36, rel=1e-13)
    # iso-surface of g_diff(k): a = -k/6, b = k/6 -> G = 0
    assert abs(od.op(2, -k / 6, k / 6)) < 1e-15
    # deep inside the left operand, the right one far outside R_o: max(a, -b)
    assert od.op(2, -0.6, 0.9) == max(-0.6, -0.9)
    # right operand deep inside: x < 0, |x| large -> K = 0 -> sharp value
    assert od.op(2, -0.05, -0.6) == pytest.approx(0.6, rel=1e-15)


@pytest.mark.parametrize("kind", [sg.SUNION, sg.SINTER, sg.SDIFF])
def test_compact_operator_continuity_at_range_boundary(kind):
    """G is continuous across a = d_o and b = d_o (the fall-back to the sharp
    operator does not jump) at d_o = 7k/6."""
    o = _op_scene(kind)
    d = o.d_o(2)
    eps = 1e-10
    for other in np.linspace(-3 * d, d, 4001):
        for (a0, b0, a1, b1) in ((d - eps, other, d + eps, other), (other, d - eps, other, d + eps)):
            assert abs(o.op(2, a0, b0) - o.op(2, a1, b1)) < 1e-8


def test_compact_union_jumps_when_d_o_equals_k():
    """The reading d_o = 7k/6 matters: with d_o = k the union jumps at the
    boundary of R_o^2.  By hand: for a = d_o, b = d_o - delta, delta > k, the
    blend radius is K = (6 delta - k)/5 > delta, so the displacement
    K/6 (1 - delta/K)^3 (about delta/1080 for large delta) survives at the
    boundary where the sharp branch has none."""
    o = _op_scene(sg.SUNION, d_o=K)
    d = o.d_o(2)
    k = float(np.float32(K))
    for delta in (2 * k, 3 * k, 3.0):
        Kb = (6 * delta - k) / 5
        jump = abs(o.op(2, d - 1e-12, d - delta) - o.op(2, d + 1e-12, d - delta))
        assert jump == pytest.approx(Kb / 6 * (1 - delta / Kb) ** 3, rel=1e-6)
    assert abs(o.op(2, d - 1e-12, d - 3.0) - o.op(2, d + 1e-12, d - 3.0)) > 2e-3


@pytest.mark.parametrize("kind,smooth", [(sg.SUNION, lambda a, b, k: min(a, b) - k / 6 * max(1 - abs(a - b) / k, 0) ** 3),
                                         (sg.SINTER, lambda a, b, k: max(a, b) + k / 6 * max(1 - abs(a - b) / k, 0) ** 3),
                                         (sg.SDIFF, lambda a, b, k: max(a, -b) + k / 6 * max(1 - abs(a + b) / k, 0) ** 3)])
def test_compact_operator_preserves_sign_of_blend(kind, smooth):
    """In isolation the compact operator keeps the 0 iso-surface of the
    unmodified blend with radius k: sign(G) = sign(g(.,.,k))."""
    o = _op_scene(kind)
    k = np.float64(np.float32(K))
    rng = np.random.default_rng(1)
    ab = rng.uniform(-0.4, 0.4, size=(20000, 2))
    for a, b in ab:
        g = smooth(a, b, k)
        G = o.op(2, a, b)
        if abs(g) > 1e-12:
            assert np.sign(G) == np.sign(g), (a, b, g, G)


@pytest.mark.parametrize("kind", [sg.SUNION, sg.SINTER, sg.SDIFF, sg.UNION, sg.INTER, sg.DIFF])
def test_operator_lipschitz_bound(kind):
    """|G(a1,b1) - G(a2,b2)| <= (1 + k/(6 d_o - k)) max(|da|, |db|) (= 7/6 for
    compact operators at d_o = 7k/6, 1 for sharp ones), sampled."""
    o = _op_scene(kind)
    bound = 7 / 6 if kind >= sg.SUNION else 1.0
    rng = np.random.default_rng(2)
    worst = 0.0
    for _ in range(40000):
        a, b = rng.uniform(-0.3, 0.3, size=2)
        da, db = rng.uniform(-1e-4, 1e-4, size=2)
        r = abs(o.op(2, a + da, b + db) - o.op(2, a, b)) / max(abs(da), abs(db))
        worst = max(worst, r)
    assert worst <= bound * (1 + 1e-6)
    if kind == sg.SUNION:
        assert worst > 1.1  # the 7/6 bound is nearly reached for the union


# ---------------------------------------------------------------------------
# Primitives and first roots: analytic ray/surface intersections.

def _pixels(cam, n=None, seed=0):
    if n is None:
        jj, ii = np.mgrid[0:cam.height, 0:cam.width]
        return (ii + 0.5).ravel().astype(float), (jj + 0.5).ravel().astype(float)
    rng = np.random.default_rng(seed)
    return rng.integers(0, cam.width, n) + 0.5, rng.integers(0, cam.height, n) + 0.5


def _quat_rot(q):
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _analytic_hit(sc, o, d):
    """First intersection of ray o + t d with the single primitive of sc, by
    ray/surface algebra (no distance field)."""
    p = sc.params[sc.root].astype(np.float64)
    k = sc.kind[sc.root]

    def sphere(c, r):
        oc = o - c
        b = oc @ d
        disc = b * b - (oc @ oc - r * r)
        if disc < 0:
            return math.inf
        t = -b - math.sqrt(disc)
        return t if t >= 0 else math.inf

    if k == sg.SPHERE:
        return sphere(p[:3], p[3])
    if k == sg.BOX:
        R = _quat_rot(p[6:10])
        ol, dl = R.T @ (o - p[:3]), R.T @ d
        lo, hi = -math.inf, math.inf
        for j in range(3):
            u, v = (-p[3 + j] - ol[j]) / dl[j], (p[3 + j] - ol[j]) / dl[j]
            lo, hi = max(lo, min(u, v)), min(hi, max(u, v))
        return lo if lo <= hi and lo >= 0 else math.inf
    if k in (sg.TORUS, sg.CYLINDER):
        # local frame of the primitive (axis of revolution = local y)
        R = _quat_rot(p[5:9])
        ol, dl = R.T @ (o - p[:3]), R.T @ d
        if k == sg.TORUS:
            return _ray_torus(ol, dl, p[3], p[4])
        return _ray_cylinder(ol, dl, p[3], p[4])
    # capsule: caps and the cylinder body between the two end planes
    a, b, r = p[:3], p[3:6], p[6]
    best = min(sphere(a, r), sphere(b, r))
    e = (b - a) / np.linalg.norm(b - a)
    L = np.linalg.norm(b - a)
    oa = o - a
    dp, op = d - (d @ e) * e, oa - (oa @ e) * e
    qa, qb, qc = dp @ dp, op @ dp, op @ op - r * r
    disc = qb * qb - qa * qc
    if disc >= 0:
        t = (-qb - math.sqrt(disc)) / qa
        s = (oa + t * d) @ e
        if 0 <= s <= L and t >= 0:
            best = min(best, t)
    return best


def _ray_torus(o, d, R, r):
    """Smallest t >= 0 with |x|^4 - 2(R^2 + r^2)|x|^2 + 4R^2 y^2 + (R^2 - r^2)^2 = 0
    (the implicit torus around the y axis, x = o + t d, |d| = 1): roots of the
    quartic, polished by Newton steps on the polynomial."""
    A, B = o @ d, o @ o + R * R - r * r
    # (t^2 + 2At + B)^2 - 4R^2((ox + t dx)^2 + (oz + t dz)^2)
    a2 = d[0] ** 2 + d[2] ** 2
    a1 = 2 * (o[0] * d[0] + o[2] * d[2])
    a0 = o[0] ** 2 + o[2] ** 2
    c = np.array([1.0, 4 * A, 4 * A * A + 2 * B - 4 * R * R * a2, 4 * A * B - 4 * R * R * a1, B * B - 4 * R * R * a0])
    best = math.inf
    for z in np.roots(c):
        if abs(z.imag) > 1e-6:
            continue
        t = z.real
        for _ in range(4):
            f, df = np.polyval(c, t), np.polyval(np.polyder(c), t)
            if df != 0:
                t -= f / df
        if t >= 0:
            best = min(best, t)
    return best


def _ray_cylinder(o, d, rad, h):
    """Smallest t >= 0 on a capped cylinder around the y axis: the side
    (x^2 + z^2 = rad^2, |y| <= h) and the two cap discs (|y| = h, x^2 + z^2 <= rad^2)."""
    best = math.inf
    qa = d[0] ** 2 + d[2] ** 2
    qb = o[0] * d[0] + o[2] * d[2]
    qc = o[0] ** 2 + o[2] ** 2 - rad * rad
    if qa > 0 and qb * qb - qa * qc >= 0:
        for sgn in (-1.0, 1.0):
            t = (-qb + sgn * math.sqrt(qb * qb - qa * qc)) / qa
            if t >= 0 and abs(o[1] + t * d[1]) <= h:
                best = min(best, t)
    if d[1] != 0:
        for y in (-h, h):
            t = (y - o[1]) / d[1]
            x, z = o[0] + t * d[0], o[2] + t * d[2]
            if t >= 0 and x * x + z * z <= rad * rad:
                best = min(best, t)
    return best


@pytest.mark.parametrize("kind", [sg.SPHERE, sg.BOX, sg.CAPSULE, sg.TORUS, sg.CYLINDER])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_first_root_matches_analytic_hit(kind, seed):
    sc = sg.single_primitive(kind, seed=seed, width=48, height=48)
    o = oracle.OracleScene(sc)
    cam = sc.camera
    px, py = _pixels(cam)
    t, nrm, flag, _ = o.trace(cam, px, py)
    eye = np.array(cam.eye, dtype=np.float64)
    nhit = 0
    for i in range(px.shape[0]):
        d = oracle.pixel_ray(cam, px[i], py[i])
        ta = _analytic_hit(sc, eye, d)
        if math.isinf(ta):
            assert not (flag[i] & 1)
        else:
            nhit += 1
            assert flag[i] & 1
            assert abs(t[i] - ta) < 1e-9
    assert nhit > 40


def test_sphere_normal_is_radial():
    sc = sg.single_primitive(sg.SPHERE, seed=3, width=40, height=40)
    o = oracle.OracleScene(sc)
    cam = sc.camera
    px, py = _pixels(cam)
    t, nrm, flag, _ = o.trace(cam, px, py)
    c, r = sc.params[sc.root, :3].astype(float), float(sc.params[sc.root, 3])
    eye = np.array(cam.eye)
    for i in np.nonzero(flag & 1)[0]:
        x = eye + t[i] * oracle.pixel_ray(cam, px[i], py[i])
        assert np.allclose(nrm[i], (x - c) / r, atol=1e-8)


@pytest.mark.parametrize("cfg_scene", ["c1", "c2", "small"])
def test_gradient_matches_central_differences(cfg_scene):
    sc = {"c1": lambda: sg.config1(1), "c2": lambda: sg.config2(1),
          "small": lambda: sg.random_small_tree(5, 7)}[cfg_scene]()
    o = oracle.OracleScene(sc)
    rng = np.random.default_rng(3)
    pts = rng.uniform(-1.2, 1.2, size=(400, 3))
    f, g = o.eval(pts, grad=True)
    h = 1e-6
    fd = np.zeros_like(g)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd[:, j] = (o.eval(pts + e) - o.eval(pts - e)) / (2 * h)
    err = np.abs(fd - g).max(axis=1)
    # kinks (sharp min/max, clamps) make a few points non-differentiable
    assert np.mean(err < 1e-6) > 0.97


@pytest.mark.parametrize("kind", [sg.SPHERE, sg.BOX, sg.CAPSULE, sg.TORUS, sg.CYLINDER])
def test_primitive_is_a_distance(kind):
    """Exact distances: |grad f| = 1 almost everywhere."""
    sc = sg.single_primitive(kind, seed=4)
    o = oracle.OracleScene(sc)
    pts = np.random.default_rng(4).uniform(-1.5, 1.5, size=(2000, 3))
    _, g = o.eval(pts, grad=True)
    assert np.mean(np.abs(np.linalg.norm(g, axis=1) - 1) < 1e-9) > 0.99


def _surface_samples(kind, p, n=200):
    """Points on the surface of a torus, capped cylinder or capped cone from
    its parametrisation (local frame, axis of revolution y), in world space."""
    th = np.linspace(0, 2 * np.pi, 4 * n, endpoint=False)
    if kind == sg.TORUS:
        ph = np.linspace(0, 2 * np.pi, n, endpoint=False)
        T, P = np.meshgrid(th, ph)
        ring = p[3] + p[4] * np.cos(P)
        loc = np.stack([ring * np.cos(T), p[4] * np.sin(P), ring * np.sin(T)], -1).reshape(-1, 3)
    elif kind == sg.CONE:
        # side: radius linear in y from p[3] at -p[4] to p[9] at +p[4]; caps: disks
        ys = np.linspace(-p[4], p[4], n)
        T, Y = np.meshgrid(th, ys)
        R = p[3] + (p[9] - p[3]) * (Y + p[4]) / (2 * p[4])
        side = np.stack([R * np.cos(T), Y, R * np.sin(T)], -1).reshape(-1, 3)
        caps = []
        for y, r in ((-p[4], p[3]), (p[4], p[9])):
            T2, RR = np.meshgrid(th, np.linspace(0, r, n // 2))
            caps.append(np.stack([RR * np.cos(T2), np.full_like(RR, y), RR * np.sin(T2)], -1).reshape(-1, 3))
        loc = np.concatenate([side] + caps)
    else:
        ys = np.linspace(-p[4], p[4], n)
        T, Y = np.meshgrid(th, ys)
        side = np.stack([p[3] * np.cos(T), Y, p[3] * np.sin(T)], -1).reshape(-1, 3)
        rr = np.linspace(0, p[3], n // 2)
        T2, RR = np.meshgrid(th, rr)
        caps = [np.stack([RR * np.cos(T2), np.full_like(RR, y), RR * np.sin(T2)], -1).reshape(-1, 3)
                for y in (-p[4], p[4])]
        loc = np.concatenate([side] + caps)
    return loc @ _quat_rot(p[5:9]).T + p[:3]


@pytest.mark.parametrize("kind", [sg.TORUS, sg.CYLINDER, sg.CONE])
def test_torus_and_cylinder_values_are_distances_to_their_surface(kind):
    """|f(x)| equals the distance from x to a dense sampling of the surface
    (parametrisation, no distance formula), within the sampling spacing, and
    f < 0 exactly where x is inside (local-frame membership test)."""
    sc = sg.single_primitive(kind, seed=6)
    o = oracle.OracleScene(sc)
    p = sc.params[sc.root].astype(np.float64)
    surf = _surface_samples(kind, p)
    spacing = 2 * np.pi * (p[3] + p[4]) / 800 + 2 * p[4] / 200
    rng = np.random.default_rng(11)
    pts = p[:3] + rng.uniform(-1.2, 1.2, size=(300, 3)) * (p[3] + p[4])
    f = o.eval(pts)
    loc = (pts - p[:3]) @ _quat_rot(p[5:9])
    rad = np.hypot(loc[:, 0], loc[:, 2])
    if kind == sg.TORUS:
        inside = (rad - p[3]) ** 2 + loc[:, 1] ** 2 < p[4] ** 2
    elif kind == sg.CONE:
        inside = (rad < p[3] + (p[9] - p[3]) * (loc[:, 1] + p[4]) / (2 * p[4])) & (np.abs(loc[:, 1]) < p[4])
    else:
        inside = (rad < p[3]) & (np.abs(loc[:, 1]) < p[4])
    for x, v, ins in zip(pts, f, inside):
        dmin = np.sqrt(((surf - x) ** 2).sum(1)).min()
        assert abs(abs(v) - dmin) <= spacing, (v, dmin)
        assert (v < 0) == ins


def test_far_union_partner_changes_nothing():
    """Sphere A compact-unioned with a sphere far away (|f_A - f_B| >> k
    wherever A's surface is) traces exactly like A alone."""
    kind = np.array([sg.SPHERE, sg.SPHERE, sg.SUNION], dtype=np.int32)
    p = np.zeros((3, 16), dtype=np.float32)
    p[0, :4] = (0.1, -0.2, 0.0, 0.6)
    p[1, :4] = (40.0, 0.0, 0.0, 0.5)
    p[2, :2] = (0.1, 0.0)
    o2 = oracle.OracleScene(kind=kind, left=np.array([-1, -1, 0], np.int32),
                            right=np.array([-1, -1, 1], np.int32), params=p, root=2)
    cam = sg.Camera(width=40, height=40)
    px, py = _pixels(cam)
    t, _, flag, _ = o2.trace(cam, px, py)
    eye = np.array(cam.eye)
    for i in range(px.shape[0]):
        d = oracle.pixel_ray(cam, px[i], py[i])
        oc = eye - p[0, :3].astype(float)
        b = oc @ d
        disc = b * b - (oc @ oc - float(p[0, 3]) ** 2)
        if disc < 0:
            assert not (flag[i] & 1)
        else:
            assert abs(t[i] - (-b - math.sqrt(disc))) < 1e-9


@pytest.mark.parametrize("make", [lambda: sg.config1(0, 24, 24), lambda: sg.random_small_tree(14, 6, width=20, height=20),
                                  lambda: sg.random_small_tree(14, 9, width=20, height=20), lambda: sg.random_small_tree(21, 6, width=20, height=20)])
def test_first_root_matches_dense_marching(make):
    """Brute force: fixed steps of 2e-4 over the full span and bisection of
    the first sign change; masks agree except on near-silhouette rays,
    depths to 1e-9."""
    sc = make()
    o = oracle.OracleScene(sc)
    cam = sc.camera
    px, py = _pixels(cam)
    t, _, flag, _ = o.trace(cam, px, py)
    tm = o.march(cam, px, py, 2e-4)
    hit, hitm = (flag & 1) != 0, np.isfinite(tm)
    near = oracle.silhouette_flags(o, cam, px, py, t, hit, 1e-4 * o.extent)
    assert np.all((hit == hitm) | near)
    both = hit & hitm & ~near
    assert both.sum() > 10
    # dense marching can land on a later root only if a sliver thinner than
    # the step exists; none does in these scenes
    assert np.max(np.abs(t[both] - tm[both])) < 1e-9


def test_camera_rays():
    cam = sg.Camera(width=101, height=61)
    d = oracle.pixel_ray(cam, 50.5, 30.5)
    assert np.allclose(d, [0, 0, -1], atol=1e-15)
    # top edge of the image (py = 0) sits at half the vertical field of view
    d = oracle.pixel_ray(cam, 50.5, 0.0)
    assert math.degrees(math.acos(-d[2])) == pytest.approx(22.5, abs=1e-12)
    assert d[1] > 0
    # right edge: tan(angle) = tan(22.5 deg) * W / H
    d = oracle.pixel_ray(cam, 101.0, 30.5)
    assert d[0] / -d[2] == pytest.approx(math.tan(math.radians(22.5)) * 101 / 61, rel=1e-12)


# ---------------------------------------------------------------------------
# Ranges and volumes of interest.

def test_range_of_interest_propagation_by_hand():
    """ROI of the root is (-inf, 0]; a compact operator hands its children
    max(d_o, d_parent), a sharp one hands them d_parent."""
    # root SUNION(k=0.1) over (SINTER(k=0.3) over (A, UNION over (B, C)), D)
    sc = sg.tree_from_shape(((0, (0, 0)), 0), [sg.UNION, sg.SINTER, sg.SUNION], k=0.3)
    sc.params[sc.root, 0] = 0.1
    o = oracle.OracleScene(sc)
    k1, k3 = float(np.float32(0.1)), float(np.float32(0.3))
    # find nodes
    root = sc.root
    inter = sc.left[root]
    d_leaf = sc.right[root]
    a, un = sc.left[inter], sc.right[inter]
    b, c = sc.left[un], sc.right[un]
    assert o.roi(root) == 0.0
    assert o.roi(inter) == pytest.approx(7 * k1 / 6, rel=1e-12)
    assert o.roi(d_leaf) == pytest.approx(7 * k1 / 6, rel=1e-12)
    assert o.roi(a) == pytest.approx(7 * k3 / 6, rel=1e-12)
    assert o.roi(un) == pytest.approx(7 * k3 / 6, rel=1e-12)
    assert o.roi(b) == pytest.approx(7 * k3 / 6, rel=1e-12)  # sharp: passes its own ROI down
    assert o.roi(c) == pytest.approx(7 * k3 / 6, rel=1e-12)


def _voi_member(sc, i, d, x):
    p = sc.params[i].astype(np.float64)
    k = sc.kind[i]
    if k == sg.SPHERE:
        return np.linalg.norm(x - p[:3]) <= p[3] + d
    if k == sg.BOX:
        return np.all(np.abs(_quat_rot(p[6:10]).T @ (x - p[:3])) <= p[3:6] + d)
    if k in (sg.TORUS, sg.CYLINDER, sg.CONE):
        r = p[3] + p[4] if k == sg.TORUS else max(p[3], p[9]) if k == sg.CONE else p[3]
        ext = np.array([r, p[4], r])
        return np.all(np.abs(_quat_rot(p[5:9]).T @ (x - p[:3])) <= ext + d)
    a, b = p[:3], p[3:6]
    s = np.clip((x - a) @ (b - a) / ((b - a) @ (b - a)), 0, 1)
    return np.linalg.norm(x - a - s * (b - a)) <= p[6] + d


@pytest.mark.parametrize("seed", [0, 1])
def test_volume_of_interest_contains_range_of_interest(seed):
    """{x : f_i(x) <= d_i} lies inside VOI_i (the bound offset by d_i), for
    every primitive type."""
    sc = sg.config2_extended(seed)
    o = oracle.OracleScene(sc)
    rng = np.random.default_rng(seed)
    prims = o.prim_ids()
    for i in prims[:60]:
        d = o.roi(i)
        c = sc.params[i, :3].astype(float)
        for x in c + rng.uniform(-0.8, 0.8, size=(300, 3)):
            if o.prim(i, x) <= d:
                assert _voi_member(sc, i, d, x)
                assert o.in_voi(i, x)


def test_field_positive_outside_every_volume_of_interest():
    """Outside all volumes of interest every primitive exceeds its range, so
    the tree value is > 0 (no surface can lie there)."""
    sc = sg.config2(2)
    o = oracle.OracleScene(sc)
    rng = np.random.default_rng(5)
    pts = rng.uniform(-1.6, 1.6, size=(3000, 3))
    f = o.eval(pts)
    prims = o.prim_ids()
    for x, v in zip(pts, f):
        if not any(o.in_voi(i, x) for i in prims):
            assert v > 0


def test_voi_intervals_are_exact():
    """Per-ray intervals: interior samples are members, samples just outside
    are not (membership computed independently)."""
    sc = sg.config2(3, width=32, height=32)
    o = oracle.OracleScene(sc)
    cam = sc.camera
    px, py = _pixels(cam, 64, seed=3)
    prims = o.prim_ids()[:40]
    z = o.voi_intervals(cam, px, py, prims)
    eye = np.array(cam.eye)
    fwd = -eye / np.linalg.norm(eye)
    checked = 0
    for r in range(px.shape[0]):
        d = oracle.pixel_ray(cam, px[r], py[r])
        cs = d @ fwd
        for q, i in enumerate(prims):
            zi, zo = z[r, q]
            if np.isnan(zi):
                continue
            t0, t1 = zi / cs, zo / cs
            for s in np.linspace(0.02, 0.98, 7):
                assert _voi_member(sc, i, o.roi(i), eye + (t0 + s * (t1 - t0)) * d)
            assert not _voi_member(sc, i, o.roi(i), eye + (t1 + 1e-6) * d)
            if t0 > 1e-6:
                assert not _voi_member(sc, i, o.roi(i), eye + (t0 - 1e-6) * d)
            checked += 1
    assert checked > 50


@pytest.mark.parametrize("make", [lambda: sg.config1(0), lambda: sg.config2(0), lambda: sg.random_small_tree(3, 8)])
def test_tree_lipschitz_bound_holds(make):
    """Sampled |f(p) - f(q)| <= L |p - q| with the product bound over
    compact levels."""
    sc = make()
    o = oracle.OracleScene(sc)
    rng = np.random.default_rng(6)
    p = rng.uniform(-1.3, 1.3, size=(50000, 3))
    q = p + rng.normal(scale=0.02, size=p.shape)
    ratio = np.abs(o.eval(p) - o.eval(q)) / np.linalg.norm(p - q, axis=1)
    assert ratio.max() <= o.lipschitz * (1 + 1e-9)


def test_lipschitz_bound_by_hand():
    """Balanced tree of 16 spheres under compact unions: 4 levels of 7/6."""
    o = oracle.OracleScene(sg.config1(0))
    assert o.lipschitz == pytest.approx((7 / 6) ** 4, rel=1e-12)
    assert o.depth == 4


def test_silhouette_ring_of_a_sphere():
    """Flagged rays of a lone sphere sit in a ring around its silhouette: every
    ray closer to it than the offset can reach along some camera axis is
    flagged, no ray far from it is."""
    sc = sg.single_primitive(sg.SPHERE, seed=7, width=64, height=64)
    o = oracle.OracleScene(sc)
    cam = sc.camera
    px, py = _pixels(cam)
    t, _, flag, _ = o.trace(cam, px, py)
    hit = (flag & 1) != 0
    off = 0.02
    # depth tolerance scaled with the offset so the slope criterion matches the
    # one used at the 1e-4 offset
    near = oracle.silhouette_flags(o, cam, px, py, t, hit, off * o.extent, offset=off)
    c, r = sc.params[sc.root, :3].astype(float), float(sc.params[sc.root, 3])
    eye = np.array(cam.eye)
    n_close = 0
    for i in range(px.shape[0]):
        d = oracle.pixel_ray(cam, px[i], py[i])
        oc = c - eye
        gap = abs(np.linalg.norm(oc - (oc @ d) * d) - r)  # ray-to-silhouette distance
        if gap > 2.5 * off:
            assert not near[i]
        if gap < 0.25 * off:
            assert near[i]
            n_close += 1
    assert n_close > 5


# ---------------------------------------------------------------------------
# MLP oracle

def test_round_half_matches_ieee_binary16():
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(scale=s, size=2000) for s in (1e-6, 1e-3, 1, 100, 3e4)])
    ref = x.astype(np.float16).astype(np.float64)  # IEEE round-to-nearest-even
    assert np.array_equal(oracle.round_half(x), ref)


def test_mlp_backward_matches_finite_differences():
    """Gradient of the FP64 loss (internal binary16 roundings off) against
    central differences, h = 1e-6."""
    rng = np.random.default_rng(8)
    W = rng.normal(scale=0.4, size=1377)
    X = rng.normal(size=(16, 8))
    T = rng.uniform(1, 4, size=16)
    for over in (4.0, 16.0):
        loss, om, g = oracle.mlp(W, X, T, exact=True, over_weight=over)
        assert om.min() >= 1 and om.max() <= 4
        for j in rng.choice(1377, 200, replace=False):
            e = np.zeros(1377)
            e[j] = 1e-6
            fd = (oracle.mlp(W + e, X, T, grad=False, exact=True, over_weight=over)[0]
                  - oracle.mlp(W - e, X, T, grad=False, exact=True, over_weight=over)[0]) / 2e-6
            assert abs(fd - g[j]) <= 1e-7 * max(1.0, abs(g[j])), (over, j)


def test_mlp_rounding_points_are_small_perturbations():
    """With the binary16 rounding points on, outputs and gradients move by
    no more than binary16 precision allows."""
    rng = np.random.default_rng(9)
    W = oracle.round_half(rng.normal(scale=0.3, size=1377))
    X = oracle.round_half(rng.normal(size=(64, 8)))
    T = rng.uniform(1, 4, size=64)
    l0, om0, g0 = oracle.mlp(W, X, T, exact=True)
    l1, om1, g1 = oracle.mlp(W, X, T)
    assert np.max(np.abs(om1 - om0)) < 1e-2
    assert np.linalg.norm(g1 - g0) < 2e-2 * np.linalg.norm(g0)


def test_mlp_forward_hand_example():
    """Zero weights: omega = 1 + 3 sigmoid(0) = 2.5 for every input."""
    W = np.zeros(1377)
    loss, om, g = oracle.mlp(W, np.ones((3, 8)), np.array([2.5, 2.0, 3.0]))
    assert np.allclose(om, 2.5)
    # loss = mean(w (omega - t)^2): (0 + 4 * 0.25 + 1 * 0.25) / 3
    assert loss == pytest.approx((0 + 4 * 0.25 + 0.25) / 3, rel=1e-15)
    # the over-prediction weight scales only the terms with omega > t
    loss16, _, _ = oracle.mlp(W, np.ones((3, 8)), np.array([2.5, 2.0, 3.0]), over_weight=16.0)
    assert loss16 == pytest.approx((0 + 16 * 0.25 + 0.25) / 3, rel=1e-15)


# ---------------------------------------------------------------------------
# Sharp-crease flag.  Normals are exempt from the parity check only where the
# field's gradient direction is not unique: two operands of a sharp branch
# (a sharp CSG node, or a compact node outside its operator range) are equal
# there.  Two spheres of radius 0.5 at (0,0,0) and (0.3,0,0) meet on the
# analytic circle x = 0.15, y^2 + z^2 = 0.25 - 0.15^2.

def _crease_circle(phi):
    r = math.sqrt(0.25 - 0.15 ** 2)
    return np.array([0.15, r * math.cos(phi), r * math.sin(phi)])


def _on_sphere(centre, radius, x):
    """The point of the sphere surface at x-coordinate x (y > 0, z = 0)."""
    y = math.sqrt(radius ** 2 - (x - centre[0]) ** 2)
    return np.array([x, y, 0.0])


@pytest.mark.parametrize("kind", [sg.UNION, sg.INTER, sg.DIFF])
def test_crease_flag_on_the_analytic_crease_circle(kind):
    o = _op_scene(kind)
    c1 = float(np.float32(0.3))
    for phi in np.linspace(0.1, 2 * math.pi, 9):
        x = _crease_circle(phi)
        x[0] = 0.5 * c1          # the bisector plane of the float32 centres
        x[1:] *= math.sqrt(0.25 - x[0] ** 2) / np.linalg.norm(x[1:])
        assert o.crease_at(x), (kind, phi)


def test_crease_flag_off_the_crease_on_each_surface():
    """A surface point 1e-3 away from the crease circle is not a crease."""
    c1 = float(np.float32(0.3))
    # union: on the outer part of sphere 0 (x < 0.15) and of sphere 1 (x > 0.15)
    o = _op_scene(sg.UNION)
    assert not o.crease_at(_on_sphere((0, 0, 0), 0.5, 0.5 * c1 - 1e-3))
    assert not o.crease_at(_on_sphere((c1, 0, 0), 0.5, 0.5 * c1 + 1e-3))
    # intersection: on the inner parts
    o = _op_scene(sg.INTER)
    assert not o.crease_at(_on_sphere((c1, 0, 0), 0.5, 0.5 * c1 - 1e-3))
    assert not o.crease_at(_on_sphere((0, 0, 0), 0.5, 0.5 * c1 + 1e-3))
    # difference sphere0 \ sphere1: the outer part of sphere 0, and the part of
    # sphere 1 inside sphere 0
    o = _op_scene(sg.DIFF)
    assert not o.crease_at(_on_sphere((0, 0, 0), 0.5, 0.5 * c1 - 1e-3))
    assert not o.crease_at(_on_sphere((c1, 0, 0), 0.5, 0.5 * c1 - 1e-3))


@pytest.mark.parametrize("kind", [sg.SUNION, sg.SINTER, sg.SDIFF])
def test_crease_flag_never_on_a_compact_blend(kind):
    """Inside the operator range the compact operators blend (C1 field): the
    crease circle of the two spheres is no crease of the blended field."""
    o = _op_scene(kind)
    c1 = float(np.float32(0.3))
    for phi in np.linspace(0.1, 2 * math.pi, 9):
        x = _crease_circle(phi)
        x[0] = 0.5 * c1
        assert not o.crease_at(x), (kind, phi)


def test_crease_flag_of_a_compact_operator_outside_its_range():
    """Outside R_o a compact union is the sharp min: equal operands there are
    a crease (points of the bisector plane far from both spheres)."""
    o = _op_scene(sg.SUNION)
    c1 = float(np.float32(0.3))
    assert o.crease_at(np.array([0.5 * c1, 0.0, 2.0]))
    assert not o.crease_at(np.array([0.5 * c1 + 1e-3, 0.0, 2.0]))


def test_crease_flag_uses_the_negated_right_operand_of_a_difference():
    """Union of C with (A \\ B) at a point of C's surface where A and B are
    equally far (a = b > 0): the difference node compares a with -b, which
    differ by 2a, so nothing is a crease there; a walk comparing a with b
    would flag it."""
    kind = np.array([sg.SPHERE, sg.SPHERE, sg.DIFF, sg.SPHERE, sg.UNION], dtype=np.int32)
    left = np.array([-1, -1, 0, -1, 3], dtype=np.int32)
    right = np.array([-1, -1, 1, -1, 2], dtype=np.int32)
    p = np.zeros((5, 16), dtype=np.float32)
    p[0, :4] = (-0.25, 0, 0, 0.2)
    p[1, :4] = (0.25, 0, 0, 0.2)
    p[3, :4] = (0, 0.75, 0, 0.25)
    o = oracle.OracleScene(kind=kind, left=left, right=right, params=p, root=4)
    x = np.array([0.0, 0.5, 0.0])          # on C's surface, on the bisector of A and B
    assert abs(o.eval(x[None])[0]) < 1e-7
    assert not o.crease_at(x)
    # and the difference's own crease (A's surface meets B's) is flagged
    o2 = oracle.OracleScene(kind=kind[:3], left=left[:3], right=right[:3], params=p[:3], root=2)
    assert not o2.crease_at(np.array([-0.45, 0.0, 0.0]))


# ---------------------------------------------------------------------------
# Scene extent (the unit of the depth tolerance): the largest edge of the
# axis-aligned box of the primitives themselves, not of their volumes of
# interest.

def test_scene_extent_by_hand_for_a_rotated_box_and_a_capsule():
    c8, s8 = math.cos(math.pi / 8), math.sin(math.pi / 8)
    kind = np.array([sg.BOX, sg.CAPSULE, sg.SUNION], dtype=np.int32)
    left = np.array([-1, -1, 0], dtype=np.int32)
    right = np.array([-1, -1, 1], dtype=np.int32)
    p = np.zeros((3, 16), dtype=np.float32)
    p[0, :10] = (0.1, -0.2, 0.05, 0.2, 0.1, 0.3, c8, 0, 0, s8)   # 45 degrees about z
    p[1, :7] = (1.0, 0.0, 0.0, 1.5, 0.5, 0.0, 0.1)
    p[2, :2] = (0.1, 0.0)
    o = oracle.OracleScene(kind=kind, left=left, right=right, params=p, root=2)
    # box: half extents along x and y (0.2 + 0.1)/sqrt(2), along z 0.3
    hxy = 0.3 / math.sqrt(2)
    x_lo, x_hi = 0.1 - hxy, 1.5 + 0.1
    y_lo, y_hi = -0.2 - hxy, 0.5 + 0.1
    z_lo, z_hi = 0.05 - 0.3, 0.05 + 0.3
    want = max(x_hi - x_lo, y_hi - y_lo, z_hi - z_lo)
    assert want == pytest.approx(1.5 + 0.1 - 0.1 + hxy)
    assert o.extent == pytest.approx(want, abs=2e-6)
    # the volumes of interest are larger: the box's local half extents and
    # the capsule's radius grow by the operator range d = 7k/6, so along x
    # the box side moves by 2d/sqrt(2) and the capsule side by d
    d = 7 * float(np.float32(0.1)) / 6
    lo, hi = o.voi_box()
    assert (hi - lo).max() == pytest.approx((1.5 + 0.1 + d) - (0.1 - (0.3 + 2 * d) / math.sqrt(2)), abs=2e-6)
    assert o.extent < (hi - lo).max() - 0.2


def test_scene_extent_of_a_lone_rotated_box():
    """A box rotated 45 degrees about z: its x edge is (h0 + h1) sqrt(2), not 2 h0."""
    c8, s8 = math.cos(math.pi / 8), math.sin(math.pi / 8)
    kind = np.array([sg.BOX], dtype=np.int32)
    p = np.zeros((1, 16), dtype=np.float32)
    p[0, :10] = (0, 0, 0, 0.5, 0.1, 0.1, c8, 0, 0, s8)
    o = oracle.OracleScene(kind=kind, left=np.array([-1], np.int32), right=np.array([-1], np.int32), params=p, root=0)
    assert o.extent == pytest.approx(0.6 * math.sqrt(2), abs=2e-6)


def _one_cone(rb, rt, h, c=(0.1, -0.2, 0.05), q=(0.9, 0.3, -0.2, 0.25)):
    """A scene of one capped cone with the given radii and half height."""
    b = sg._Builder()
    qq = np.asarray(q, dtype=np.float64)
    qq = qq / np.linalg.norm(qq)
    root = b.add(sg.CONE, p=(*c, rb, h, *qq, rt))
    return b.finish("one_cone", root, sg.Camera(width=32, height=32), {"config": 0, "seed": 0, "tile": 8})


def test_cone_with_equal_radii_is_the_cylinder():
    """A cone whose two radii are equal is the capped cylinder of that radius
    (the cylinder's own pins fix that one)."""
    cone = _one_cone(0.4, 0.4, 0.3)
    b = sg._Builder()
    pc = cone.params[cone.root].astype(np.float64)
    root = b.add(sg.CYLINDER, p=(*pc[:3], pc[3], pc[4], *pc[5:9]))
    cyl = b.finish("one_cyl", root, sg.Camera(width=32, height=32), {"config": 0, "seed": 0, "tile": 8})
    rng = np.random.default_rng(3)
    pts = pc[:3] + rng.uniform(-0.9, 0.9, size=(500, 3))
    fa = oracle.OracleScene(cone).eval(pts)
    fb = oracle.OracleScene(cyl).eval(pts)
    assert np.allclose(fa, fb, rtol=0, atol=1e-12)


@pytest.mark.parametrize("rb,rt", [(0.5, 0.0), (0.0, 0.4), (0.5, 0.2)])
def test_cone_closed_forms_on_its_axis(rb, rt):
    """On the axis: beyond a cap the distance is the height above that cap's
    plane; inside, minus the smaller of the distance to the nearer cap plane
    and the perpendicular distance to the side line (for a point on the axis
    its foot falls on the side segment here)."""
    sc = _one_cone(rb, rt, 0.3)
    p = sc.params[sc.root].astype(np.float64)
    rb, h, rt = p[3], p[4], p[9]   # as stored (float32)
    R = _quat_rot(p[5:9])
    axis = R[:, 1]
    L = np.hypot(rt - rb, 2 * h)
    for y in (-0.9, -0.5, -0.31, 0.31, 0.5, 0.9, -0.2, -0.05, 0.0, 0.1, 0.25):
        x = p[:3] + y * axis
        f = oracle.OracleScene(sc).eval(x[None, :])[0]
        if abs(y) > h:
            want = abs(y) - h
        else:
            side = abs((0 - rb) * 2 * h - (y + h) * (rt - rb)) / L
            want = -min(h - abs(y), side)
        assert abs(f - want) < 1e-12, (y, f, want)


def test_cone_gradient_has_unit_norm():
    """The value is a Euclidean distance: its forward-mode gradient has norm 1
    away from the medial axis (where it jumps) and equals central differences
    of the value."""
    sc = _one_cone(0.45, 0.15, 0.35)
    o = oracle.OracleScene(sc)
    p = sc.params[sc.root].astype(np.float64)
    rng = np.random.default_rng(5)
    pts = p[:3] + rng.uniform(-0.8, 0.8, size=(200, 3))
    f, g = o.eval(pts, grad=True)
    e = 1e-6
    cd = np.stack([(o.eval(pts + e * u) - o.eval(pts - e * u)) / (2 * e) for u in np.eye(3)], -1)
    smooth = np.abs(np.linalg.norm(cd, axis=1) - 1) < 1e-4   # off the medial axis
    assert smooth.sum() >= 190
    assert np.allclose(np.linalg.norm(g[smooth], axis=1), 1, atol=1e-9)
    assert np.allclose(g[smooth], cd[smooth], atol=1e-5)
