/*
 * FP64 CPU oracle for synchronized tracing of blobtrees (Zanni 2023,
 * "Synchronized-tracing of implicit surfaces").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no source with the GPU path.
 *
 * What it computes, plainly and slowly, in double precision:
 *   - the FULL blobtree field f (no pruning, no A-buffer), recursively, and its
 *     gradient by forward-mode differentiation;
 *   - the first root t* of f along each pixel ray, its hit/miss status and the
 *     unit normal grad f / |grad f| at t*;
 *   - ranges of interest, volumes of interest and brute-force per-ray
 *     volume-of-interest intervals (what a tile A-buffer must cover);
 *   - a silhouette flag per ray (four parallel rays offset by 1e-4);
 *   - an FP64 forward/backward of the step-predictor MLP.
 *
 * Parity status of each function is stated where it is defined; the pins live
 * in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    K_SPHERE = 0, K_BOX = 1, K_CAPSULE = 2, K_TORUS = 3, K_CYLINDER = 4, K_CONE = 5,
    K_UNION = 16, K_INTER = 17, K_DIFF = 18,
    K_SUNION = 19, K_SINTER = 20, K_SDIFF = 21
};

typedef struct {
    int n, root;
    int *kind, *left, *right;
    double *par;       /* n x 16, primitives: as given; boxes: + rotation */
    double *rot;       /* n x 9, box rotation matrices (columns = box axes) */
    double *kk, *dop;  /* blend radius k and operator range d_o per operator */
    double *roi;       /* upper end d of each node's range of interest */
    double lip;        /* Lipschitz bound of the whole tree */
    int depth;         /* longest root-to-leaf edge count */
    double voi_lo[3], voi_hi[3];  /* AABB of all volumes of interest */
    double ext_lo[3], ext_hi[3];  /* AABB of all primitives (scene extent) */
} or_scene;

static int is_prim(int k) { return k >= K_SPHERE && k <= K_CONE; }
/* primitives with a rotated local frame: the box (quaternion at p[6..9]),
 * the torus and the cylinder (quaternion at p[5..8]) */
static int quat_offset(int k) { return k == K_BOX ? 6 : (k == K_TORUS || k == K_CYLINDER || k == K_CONE) ? 5 : -1; }
static int is_op(int k) { return k >= K_UNION && k <= K_SDIFF; }
static int is_compact(int k) { return k >= K_SUNION && k <= K_SDIFF; }

/* ------------------------------------------------------------------------ */
/* Forward-mode dual numbers: value and gradient with respect to the point.  */
typedef struct { double v, g[3]; } dual;

static dual dconst(double c) { dual r = {c, {0, 0, 0}}; return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int i = 0; i < 3; i++) r.g[i] = a.g[i] + b.g[i]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int i = 0; i < 3; i++) r.g[i] = a.g[i] - b.g[i]; return r; }
static dual dneg(dual a) { dual r; r.v = -a.v; for (int i = 0; i < 3; i++) r.g[i] = -a.g[i]; return r; }
static dual dmul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int i = 0; i < 3; i++) r.g[i] = a.g[i] * b.v + a.v * b.g[i]; return r; }
static dual dscale(dual a, double s) { dual r; r.v = a.v * s; for (int i = 0; i < 3; i++) r.g[i] = a.g[i] * s; return r; }
static dual ddiv(dual a, dual b) { dual r; r.v = a.v / b.v; for (int i = 0; i < 3; i++) r.g[i] = (a.g[i] * b.v - a.v * b.g[i]) / (b.v * b.v); return r; }
static dual dabs(dual a) { return a.v < 0 ? dneg(a) : a; }
static dual dmin(dual a, dual b) { return b.v < a.v ? b : a; }
static dual dmax(dual a, dual b) { return b.v > a.v ? b : a; }
static dual dsqrt(dual a) {
    dual r; r.v = sqrt(a.v);
    for (int i = 0; i < 3; i++) r.g[i] = r.v > 0 ? a.g[i] / (2 * r.v) : 0;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Primitives: exact Euclidean signed distances (Lipschitz 1).  The paper
 * assumes well-behaved primitives of Lipschitz bound <= 1 (Section
 * "Primitive volume of interest"); the formulas are the textbook ones. */

static void quat_to_rot(const double q_in[4], double R[9]) {
    double w = q_in[0], x = q_in[1], y = q_in[2], z = q_in[3];
    double n = sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    /* R is row-major; its columns are the images of the local axes. */
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static dual prim_dual(const or_scene *s, int i, const dual p[3]) {
    const double *a = s->par + 16 * i;
    switch (s->kind[i]) {
    case K_SPHERE: {
        dual d[3]; for (int j = 0; j < 3; j++) d[j] = dsub(p[j], dconst(a[j]));
        dual len = dsqrt(dadd(dadd(dmul(d[0], d[0]), dmul(d[1], d[1])), dmul(d[2], d[2])));
        return dsub(len, dconst(a[3]));
    }
    case K_BOX: {
        const double *R = s->rot + 9 * i;
        dual d[3]; for (int j = 0; j < 3; j++) d[j] = dsub(p[j], dconst(a[j]));
        dual q[3];
        for (int j = 0; j < 3; j++) {   /* local = R^T (p - c) */
            q[j] = dadd(dadd(dscale(d[0], R[0 * 3 + j]), dscale(d[1], R[1 * 3 + j])), dscale(d[2], R[2 * 3 + j]));
            q[j] = dsub(dabs(q[j]), dconst(a[3 + j]));
        }
        dual o2 = dconst(0);
        for (int j = 0; j < 3; j++) { dual m = dmax(q[j], dconst(0)); o2 = dadd(o2, dmul(m, m)); }
        dual outside = dsqrt(o2);
        dual inside = dmin(dmax(dmax(q[0], q[1]), q[2]), dconst(0));
        return dadd(outside, inside);
    }
    case K_CAPSULE: {
        dual pa[3]; double ba[3], bb = 0;
        for (int j = 0; j < 3; j++) { pa[j] = dsub(p[j], dconst(a[j])); ba[j] = a[3 + j] - a[j]; bb += ba[j] * ba[j]; }
        dual h = dconst(0);
        if (bb > 0) {
            h = dscale(dadd(dadd(dscale(pa[0], ba[0]), dscale(pa[1], ba[1])), dscale(pa[2], ba[2])), 1.0 / bb);
            h = dmin(dmax(h, dconst(0)), dconst(1));
        }
        dual w2 = dconst(0);
        for (int j = 0; j < 3; j++) { dual w = dsub(pa[j], dscale(h, ba[j])); w2 = dadd(w2, dmul(w, w)); }
        return dsub(dsqrt(w2), dconst(a[6]));
    }
    case K_TORUS:
    case K_CYLINDER: {
        /* local coordinates l = R^T (p - c); the axis of revolution is local y.
         * Torus (ring of major radius a[3] in the local x-z plane, tube radius
         * a[4]): distance | (sqrt(lx^2 + lz^2) - a[3], ly) | - a[4].
         * Capped cylinder (radius a[3], half height a[4]): with
         * w = (sqrt(lx^2 + lz^2) - a[3], |ly| - a[4]), the distance is
         * |max(w, 0)| + min(max(w.x, w.y), 0). */
        const double *R = s->rot + 9 * i;
        dual d[3]; for (int j = 0; j < 3; j++) d[j] = dsub(p[j], dconst(a[j]));
        dual l[3];
        for (int j = 0; j < 3; j++)
            l[j] = dadd(dadd(dscale(d[0], R[0 * 3 + j]), dscale(d[1], R[1 * 3 + j])), dscale(d[2], R[2 * 3 + j]));
        dual rad = dsqrt(dadd(dmul(l[0], l[0]), dmul(l[2], l[2])));
        if (s->kind[i] == K_TORUS) {
            dual qx = dsub(rad, dconst(a[3]));
            return dsub(dsqrt(dadd(dmul(qx, qx), dmul(l[1], l[1]))), dconst(a[4]));
        }
        dual wx = dsub(rad, dconst(a[3])), wy = dsub(dabs(l[1]), dconst(a[4]));
        dual ox = dmax(wx, dconst(0)), oy = dmax(wy, dconst(0));
        dual outside = dsqrt(dadd(dmul(ox, ox), dmul(oy, oy)));
        return dadd(outside, dmin(dmax(wx, wy), dconst(0)));
    }
    case K_CONE: {
        /* Capped cone: axis local y, bottom disk radius a[3] at y = -a[4], top
         * disk radius a[9] at y = +a[4].  In the meridian half-plane (rho, y),
         * rho = sqrt(lx^2 + lz^2), the solid is the trapezoid bounded by the
         * two cap segments and the side segment S from (a[3], -a[4]) to
         * (a[9], a[4]).  Distance to the surface: the smaller of the distance
         * to the cap segment on the point's side of y = 0 and the distance to
         * S (closest point at the clamped projection parameter); negative
         * inside, which is |y| < a[4] and the point left of S. */
        const double *R = s->rot + 9 * i;
        dual d[3]; for (int j = 0; j < 3; j++) d[j] = dsub(p[j], dconst(a[j]));
        dual l[3];
        for (int j = 0; j < 3; j++)
            l[j] = dadd(dadd(dscale(d[0], R[0 * 3 + j]), dscale(d[1], R[1 * 3 + j])), dscale(d[2], R[2 * 3 + j]));
        const double rb = a[3], h = a[4], rt = a[9];
        dual rho = dsqrt(dadd(dmul(l[0], l[0]), dmul(l[2], l[2])));
        const double rcap = l[1].v < 0 ? rb : rt;
        dual cax = dsub(rho, dmin(rho, dconst(rcap)));
        dual cay = dsub(dabs(l[1]), dconst(h));
        const double ex = rt - rb, ey = 2 * h, ee = ex * ex + ey * ey;
        dual px = dsub(rho, dconst(rb)), py = dadd(l[1], dconst(h));     /* point relative to the bottom end of S */
        dual tt = dscale(dadd(dscale(px, ex), dscale(py, ey)), 1.0 / ee);
        tt = dmin(dmax(tt, dconst(0)), dconst(1));
        dual cbx = dsub(px, dscale(tt, ex)), cby = dsub(py, dscale(tt, ey));
        dual dcap = dadd(dmul(cax, cax), dmul(cay, cay)), dside = dadd(dmul(cbx, cbx), dmul(cby, cby));
        dual dist = dsqrt(dmin(dcap, dside));
        /* left of S: the cross product of S's direction and the point is positive */
        const int inside = cay.v < 0 && (ex * py.v - ey * px.v) > 0;
        return inside ? dneg(dist) : dist;
    }
    }
    return dconst(INFINITY);
}

/* Half extents of the local box of a torus or cylinder (local x, y, z). */
static void ring_extents(const or_scene *s, int i, double e[3]) {
    const double *a = s->par + 16 * i;
    if (s->kind[i] == K_TORUS) { e[0] = e[2] = a[3] + a[4]; e[1] = a[4]; }
    else if (s->kind[i] == K_CONE) { e[0] = e[2] = fmax(a[3], a[9]); e[1] = a[4]; }
    else { e[0] = e[2] = a[3]; e[1] = a[4]; }
}

/* ------------------------------------------------------------------------ */
/* Operators.
 * Sharp CSG: eq. (union), (intersect), (diff): min, max, max(f0, -f1).
 * Polynomial C2 smooth operators: eq. (smooth-union)...(smooth-diff) with the
 *   displacement d(f0,f1,k) = k/6 max(1 - |f0-f1|/k, 0)^3 (eq. disp_smooth).
 * Compact operators, eq. (smooth_comp): the local operator gbar when both
 *   operands lie in R_o = (-inf, d_o], the sharp operator otherwise; gbar
 *   evaluates g twice, the first time to interpolate the blend radius with
 *   b_r(x,k,d) = k max(1 - 6x/(6d-k), 0) (eq. compact_smooth_union).
 * Readings taken where the text is loose:
 *   - a blend radius K <= 0 gives zero displacement (the "not a number" of
 *     the text is filtered by this guard, never by fmax semantics);
 *   - the upper bound K <= k applies to intersection and difference only;
 *   - for the difference the absolute value is applied to the argument of
 *     b_r (b_r itself is never negative);
 *   - R_o is closed and the right operand of a difference is tested as
 *     f1 <= d_o;
 *   - d_o <= 0 in the input means d_o = 7k/6, the smallest value for which the
 *     union stays continuous across the boundary of R_o^2.
 */
static dual disp(dual a, dual b, dual K) {
    if (!(K.v > 0)) return dconst(0);
    dual h = dsub(dconst(1), ddiv(dabs(dsub(a, b)), K));
    if (h.v <= 0) return dconst(0);
    return dmul(dscale(K, 1.0 / 6.0), dmul(h, dmul(h, h)));
}
static dual g_union(dual a, dual b, dual K) { return dsub(dmin(a, b), disp(a, b, K)); }
static dual g_inter(dual a, dual b, dual K) { return dadd(dmax(a, b), disp(a, b, K)); }
static dual g_diff(dual a, dual b, dual K) { return dadd(dmax(a, dneg(b)), disp(a, dneg(b), K)); }

static dual b_r(dual x, double k, double d) {
    dual t = dsub(dconst(1), dscale(x, 6.0 / (6.0 * d - k)));
    if (t.v <= 0) return dconst(0);
    return dscale(t, k);
}

static dual op_dual(const or_scene *s, int i, dual a, dual b) {
    double k = s->kk[i], d = s->dop[i];
    switch (s->kind[i]) {
    case K_UNION: return dmin(a, b);
    case K_INTER: return dmax(a, b);
    case K_DIFF: return dmax(a, dneg(b));
    case K_SUNION:
        if (a.v <= d && b.v <= d) {
            dual K = b_r(g_union(a, b, dconst(k)), k, d);
            return g_union(a, b, K);
        }
        return dmin(a, b);
    case K_SINTER:
        if (a.v <= d && b.v <= d) {
            dual K = dmin(b_r(g_inter(a, b, dconst(k)), k, d), dconst(k));
            return g_inter(a, b, K);
        }
        return dmax(a, b);
    case K_SDIFF:
        if (a.v <= d && b.v <= d) {
            dual K = dmin(b_r(dabs(g_diff(a, b, dconst(k))), k, d), dconst(k));
            return g_diff(a, b, K);
        }
        return dmax(a, dneg(b));
    }
    return dconst(INFINITY);
}

/* Full-tree field, recursive (no pruning).  Parity pinned by the primitive,
 * operator and first-root tests. */
static dual node_dual(const or_scene *s, int i, const dual p[3]) {
    if (is_prim(s->kind[i])) return prim_dual(s, i, p);
    dual a = node_dual(s, s->left[i], p);
    dual b = node_dual(s, s->right[i], p);
    return op_dual(s, i, a, b);
}

static double field(const or_scene *s, const double x[3], double grad[3]) {
    dual p[3];
    for (int j = 0; j < 3; j++) { p[j] = dconst(x[j]); p[j].g[j] = 1; }
    dual r = node_dual(s, s->root, p);
    if (grad) for (int j = 0; j < 3; j++) grad[j] = r.g[j];
    return r.v;
}

/* ------------------------------------------------------------------------ */
/* Scene construction: validation, d_o, ranges of interest (propagated from
 * the root, whose range is (-inf, 0]; a compact node hands its children
 * max(d_o, d_parent), a sharp node hands them d_parent), Lipschitz bound. */

static void aabb_add(double lo[3], double hi[3], const double a[3], const double b[3]) {
    for (int j = 0; j < 3; j++) { if (a[j] < lo[j]) lo[j] = a[j]; if (b[j] > hi[j]) hi[j] = b[j]; }
}

/* Axis-aligned box of primitive i grown by offset d (d = 0: the primitive;
 * d = its ROI: its volume of interest). */
static void prim_aabb(const or_scene *s, int i, double d, double lo[3], double hi[3]) {
    const double *a = s->par + 16 * i;
    switch (s->kind[i]) {
    case K_SPHERE:
        for (int j = 0; j < 3; j++) { lo[j] = a[j] - a[3] - d; hi[j] = a[j] + a[3] + d; }
        break;
    case K_BOX: {
        const double *R = s->rot + 9 * i;
        for (int j = 0; j < 3; j++) {
            double e = 0;
            for (int c = 0; c < 3; c++) e += fabs(R[j * 3 + c]) * (a[3 + c] + d);
            lo[j] = a[j] - e; hi[j] = a[j] + e;
        }
        break;
    }
    case K_CAPSULE:
        for (int j = 0; j < 3; j++) {
            double m = fmin(a[j], a[3 + j]), M = fmax(a[j], a[3 + j]);
            lo[j] = m - a[6] - d; hi[j] = M + a[6] + d;
        }
        break;
    case K_TORUS:
    case K_CYLINDER:
    case K_CONE: {
        const double *R = s->rot + 9 * i;
        double ext[3];
        ring_extents(s, i, ext);
        for (int j = 0; j < 3; j++) {
            double e = 0;
            for (int c = 0; c < 3; c++) e += fabs(R[j * 3 + c]) * (ext[c] + d);
            lo[j] = a[j] - e; hi[j] = a[j] + e;
        }
        break;
    }
    }
}

void or_scene_free(or_scene *s) {
    if (!s) return;
    free(s->kind); free(s->left); free(s->right); free(s->par); free(s->rot);
    free(s->kk); free(s->dop); free(s->roi); free(s);
}

/* Returns NULL on a malformed tree or parameters. */
or_scene *or_scene_new(const int32_t *kind, const int32_t *left, const int32_t *right,
                       const float *params, int n, int root) {
    if (n <= 0 || root < 0 || root >= n) return NULL;
    or_scene *s = (or_scene *)calloc(1, sizeof(or_scene));
    s->n = n; s->root = root;
    s->kind = (int *)malloc(sizeof(int) * n); s->left = (int *)malloc(sizeof(int) * n);
    s->right = (int *)malloc(sizeof(int) * n);
    s->par = (double *)calloc((size_t)16 * n, sizeof(double));
    s->rot = (double *)calloc((size_t)9 * n, sizeof(double));
    s->kk = (double *)calloc(n, sizeof(double)); s->dop = (double *)calloc(n, sizeof(double));
    s->roi = (double *)calloc(n, sizeof(double));
    for (int i = 0; i < n; i++) {
        s->kind[i] = kind[i]; s->left[i] = left[i]; s->right[i] = right[i];
        for (int j = 0; j < 16; j++) s->par[16 * i + j] = (double)params[16 * i + j];
        if (!is_prim(kind[i]) && !is_op(kind[i])) goto bad;
        if (is_op(kind[i]) && (left[i] < 0 || left[i] >= n || right[i] < 0 || right[i] >= n)) goto bad;
        if (quat_offset(kind[i]) >= 0) quat_to_rot(s->par + 16 * i + quat_offset(kind[i]), s->rot + 9 * i);
        if (is_compact(kind[i])) {
            double k = s->par[16 * i], d = s->par[16 * i + 1];
            if (!(k > 0)) goto bad;
            if (!(d > 0)) d = 7.0 * k / 6.0;
            if (!(6 * d - k > 0)) goto bad;
            s->kk[i] = k; s->dop[i] = d;
        }
    }
    /* iterative walk from the root: every node visited once, ROI and depth */
    {
        int *stack = (int *)malloc(sizeof(int) * (n + 1)), *dep = (int *)calloc(n, sizeof(int));
        char *seen = (char *)calloc(n, 1);
        double *lip = (double *)calloc(n, sizeof(double));
        int sp = 0, cnt = 0, maxd = 0;
        stack[sp++] = root; s->roi[root] = 0.0; lip[root] = 1.0;
        for (int j = 0; j < 3; j++) {
            s->voi_lo[j] = s->ext_lo[j] = INFINITY; s->voi_hi[j] = s->ext_hi[j] = -INFINITY;
        }
        double L = 1.0;
        while (sp) {
            int i = stack[--sp];
            if (seen[i]) { free(stack); free(dep); free(seen); free(lip); goto bad; }
            seen[i] = 1; cnt++;
            if (dep[i] > maxd) maxd = dep[i];
            if (is_op(s->kind[i])) {
                double dc = s->roi[i], f = lip[i];
                if (is_compact(s->kind[i])) {
                    if (s->dop[i] > dc) dc = s->dop[i];
                    f *= 1.0 + s->kk[i] / (6.0 * s->dop[i] - s->kk[i]);
                }
                int c[2] = {s->left[i], s->right[i]};
                for (int q = 0; q < 2; q++) {
                    s->roi[c[q]] = dc; dep[c[q]] = dep[i] + 1; lip[c[q]] = f;
                    stack[sp++] = c[q];
                    if (sp > n) { free(stack); free(dep); free(seen); free(lip); goto bad; }
                }
            } else {
                double lo[3], hi[3];
                if (lip[i] > L) L = lip[i];
                prim_aabb(s, i, 0.0, lo, hi); aabb_add(s->ext_lo, s->ext_hi, lo, hi);
                prim_aabb(s, i, s->roi[i], lo, hi); aabb_add(s->voi_lo, s->voi_hi, lo, hi);
            }
        }
        free(stack); free(dep); free(seen); free(lip);
        if (cnt != n) goto bad;
        s->depth = maxd; s->lip = L;
    }
    return s;
bad:
    or_scene_free(s);
    return NULL;
}

double or_scene_lipschitz(const or_scene *s) { return s->lip; }
int or_scene_depth(const or_scene *s) { return s->depth; }
double or_scene_roi(const or_scene *s, int i) { return s->roi[i]; }
double or_scene_dop(const or_scene *s, int i) { return s->dop[i]; }
double or_scene_extent(const or_scene *s) {
    double e = 0;
    for (int j = 0; j < 3; j++) e = fmax(e, s->ext_hi[j] - s->ext_lo[j]);
    return e;
}
void or_scene_voi_box(const or_scene *s, double lo[3], double hi[3]) {
    for (int j = 0; j < 3; j++) { lo[j] = s->voi_lo[j]; hi[j] = s->voi_hi[j]; }
}

/* Field value (and gradient when grad != NULL) at n points, full tree. */
void or_eval(const or_scene *s, const double *pts, int n, double *out_f, double *out_grad) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        double g[3];
        out_f[i] = field(s, pts + 3 * i, out_grad ? g : NULL);
        if (out_grad) for (int j = 0; j < 3; j++) out_grad[3 * i + j] = g[j];
    }
}

/* Single operator on given operand values, node i's kind and parameters
 * (used by the closed-form and continuity pins). */
double or_op(const or_scene *s, int i, double a, double b) {
    return op_dual(s, i, dconst(a), dconst(b)).v;
}

/* ------------------------------------------------------------------------ */
/* Pinhole camera: eye, target, up, vertical field of view, W x H.  Pixel
 * (i, j), row 0 at the top, has its ray through the pixel centre; t is the
 * distance along the unit direction. */
typedef struct { double eye[3], target[3], up[3], vfov_deg; int w, h; } or_camera;

static void normalize3(double v[3]) { double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); v[0] /= n; v[1] /= n; v[2] /= n; }
static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1]; c[1] = a[2] * b[0] - a[0] * b[2]; c[2] = a[0] * b[1] - a[1] * b[0];
}

static void camera_basis(const or_camera *c, double fwd[3], double right[3], double up[3]) {
    for (int j = 0; j < 3; j++) fwd[j] = c->target[j] - c->eye[j];
    normalize3(fwd);
    cross3(fwd, c->up, right); normalize3(right);
    cross3(right, fwd, up);
}

static void pixel_ray(const or_camera *c, double px, double py, double dir[3]) {
    double fwd[3], right[3], up[3];
    camera_basis(c, fwd, right, up);
    double th = tan(0.5 * c->vfov_deg * M_PI / 180.0);
    double x = (2.0 * px / c->w - 1.0) * th * ((double)c->w / c->h);
    double y = (1.0 - 2.0 * py / c->h) * th;
    for (int j = 0; j < 3; j++) dir[j] = x * right[j] + y * up[j] + fwd[j];
    normalize3(dir);
}

void or_pixel_ray(const double *cam, int w, int h, double px, double py, double dir[3]) {
    or_camera c; memcpy(c.eye, cam, 3 * sizeof(double)); memcpy(c.target, cam + 3, 3 * sizeof(double));
    memcpy(c.up, cam + 6, 3 * sizeof(double)); c.vfov_deg = cam[9]; c.w = w; c.h = h;
    pixel_ray(&c, px, py, dir);
}

/* Ray / axis-aligned box entry and exit, clipped to t >= 0. */
static int ray_aabb(const double o[3], const double d[3], const double lo[3], const double hi[3],
                    double *t0, double *t1) {
    double a = 0.0, b = INFINITY;
    for (int j = 0; j < 3; j++) {
        if (d[j] == 0.0) { if (o[j] < lo[j] || o[j] > hi[j]) return 0; continue; }
        double u = (lo[j] - o[j]) / d[j], v = (hi[j] - o[j]) / d[j];
        if (u > v) { double w = u; u = v; v = w; }
        if (u > a) a = u;
        if (v < b) b = v;
    }
    if (a > b) return 0;
    *t0 = a; *t1 = b;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* First root of f along a ray (plain definition: the smallest t >= t_a with
 * f(r(t)) <= 0, where [t_a, t_b] is the ray's span inside the box of all
 * volumes of interest; outside every volume of interest f > 0).
 *  1. sphere tracing with the proven tree Lipschitz bound (steps never cross
 *     a root) until the safe step drops below 1e-7;
 *  2. forward probing with doubling steps from 1e-7 until f <= 0 (bracket)
 *     or f stops decreasing (grazing miss: back to 1);
 *  3. bisection of the bracket to a width below 1e-12.
 * At most 10^6 field evaluations; a ray that exhausts them is "undecided".
 * Returns 1 hit, 0 miss, -1 undecided. */
#define OR_CAP 1000000

static int bisect_root(const or_scene *s, const double o[3], const double d[3],
                       double lo, double hi, double *t_out, long *evals) {
    while (hi - lo > 1e-12) {
        double m = 0.5 * (lo + hi), p[3];
        if (m <= lo || m >= hi) break;
        for (int j = 0; j < 3; j++) p[j] = o[j] + m * d[j];
        double f = field(s, p, NULL); (*evals)++;
        if (f <= 0) hi = m; else lo = m;
    }
    *t_out = hi;
    return 1;
}

static int first_root(const or_scene *s, const double o[3], const double d[3], double *t_out,
                      long *evals_out) {
    double ta, tb, p[3];
    long ev = 0;
    int res = 0;
    *t_out = INFINITY;
    if (!ray_aabb(o, d, s->voi_lo, s->voi_hi, &ta, &tb)) { *evals_out = 0; return 0; }
    double t = ta, L = s->lip;
    for (int j = 0; j < 3; j++) p[j] = o[j] + t * d[j];
    double f = field(s, p, NULL); ev++;
    if (f <= 0) { *t_out = t; *evals_out = ev; return 1; }
    while (t <= tb) {
        if (ev > OR_CAP) { res = -1; break; }
        double step = f / L;
        if (step >= 1e-7) {
            t += step;
            for (int j = 0; j < 3; j++) p[j] = o[j] + t * d[j];
            double f2 = field(s, p, NULL); ev++;
            if (f2 <= 0) {   /* a safe step landed on the surface */
                bisect_root(s, o, d, t - step, t, t_out, &ev);
                res = 1; break;
            }
            f = f2;
            continue;
        }
        /* near the surface: probe forward with doubling steps */
        double h = 1e-7;
        int found = 0;
        for (;;) {
            if (ev > OR_CAP) { res = -1; break; }
            double t2 = t + h;
            for (int j = 0; j < 3; j++) p[j] = o[j] + t2 * d[j];
            double f2 = field(s, p, NULL); ev++;
            if (f2 <= 0) { bisect_root(s, o, d, t, t2, t_out, &ev); found = 1; break; }
            int rising = f2 >= f;
            t = t2; f = f2; h *= 2;
            if (rising || t > tb) break;
        }
        if (found) { res = 1; break; }
        if (res < 0) break;
    }
    *evals_out = ev;
    return res;
}

/* Sharp-crease flag: at the hit point, some node evaluated on its sharp branch
 * (or a sharp CSG node) sees two operands closer than 1e-6, so the gradient
 * direction is not unique there. */
static int crease_walk(const or_scene *s, int i, const double x[3], double *val) {
    if (is_prim(s->kind[i])) {
        dual p[3]; for (int j = 0; j < 3; j++) p[j] = dconst(x[j]);
        *val = prim_dual(s, i, p).v;
        return 0;
    }
    double a, b;
    int c = crease_walk(s, s->left[i], x, &a) | crease_walk(s, s->right[i], x, &b);
    dual r = op_dual(s, i, dconst(a), dconst(b));
    *val = r.v;
    int k = s->kind[i];
    double bb = (k == K_DIFF || k == K_SDIFF) ? -b : b;
    int sharp_branch = !is_compact(k) || !(a <= s->dop[i] && b <= s->dop[i]);
    if (sharp_branch && fabs(a - bb) < 1e-6) c = 1;
    return c;
}

/* Crease flag of the point x (the walk above from the root).  Parity pinned
 * by analytic crease circles of two-sphere sharp operators, off-crease
 * surface points, compact blends and a nested difference. */
int or_crease_at(const or_scene *s, const double x[3]) {
    double val;
    return crease_walk(s, s->root, x, &val);
}

/* Trace the rays of pixels (px[i], py[i]) (pixel-centre coordinates, i.e.
 * col + 0.5, row + 0.5), optionally displaced parallel to themselves by
 * (off_r, off_u) along the camera right/up axes.
 * out_t: t* or +inf; out_n: unit normal (0 on miss);
 * out_flag: bit0 hit, bit1 undecided, bit2 crease at the hit;
 * out_evals: field evaluations used. */
void or_trace(const or_scene *s, const double *cam, int w, int h, const double *px, const double *py,
              int n, double off_r, double off_u, double *out_t, double *out_n, int32_t *out_flag,
              int64_t *out_evals) {
    or_camera c; memcpy(c.eye, cam, 3 * sizeof(double)); memcpy(c.target, cam + 3, 3 * sizeof(double));
    memcpy(c.up, cam + 6, 3 * sizeof(double)); c.vfov_deg = cam[9]; c.w = w; c.h = h;
    double fwd[3], right[3], up[3];
    camera_basis(&c, fwd, right, up);
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; i++) {
        double d[3], o[3], t;
        long ev = 0;
        pixel_ray(&c, px[i], py[i], d);
        for (int j = 0; j < 3; j++) o[j] = c.eye[j] + off_r * right[j] + off_u * up[j];
        int r = first_root(s, o, d, &t, &ev);
        int flag = 0;
        double nrm[3] = {0, 0, 0};
        if (r == 1) {
            double x[3], g[3], val;
            flag |= 1;
            for (int j = 0; j < 3; j++) x[j] = o[j] + t * d[j];
            field(s, x, g); ev++;
            double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            if (gn > 0) for (int j = 0; j < 3; j++) nrm[j] = g[j] / gn;
            if (crease_walk(s, s->root, x, &val)) flag |= 4;
        } else if (r < 0) {
            flag |= 2;
            t = INFINITY;
        }
        out_t[i] = r == 1 ? t : INFINITY;
        for (int j = 0; j < 3; j++) out_n[3 * i + j] = nrm[j];
        out_flag[i] = flag;
        if (out_evals) out_evals[i] = ev;
    }
}

/* Dense ray marching (pin for or_trace): fixed steps dt over the ray's span
 * in the box of all volumes of interest, first sign change bisected. */
void or_march(const or_scene *s, const double *cam, int w, int h, const double *px, const double *py,
              int n, double dt, double *out_t) {
    or_camera c; memcpy(c.eye, cam, 3 * sizeof(double)); memcpy(c.target, cam + 3, 3 * sizeof(double));
    memcpy(c.up, cam + 6, 3 * sizeof(double)); c.vfov_deg = cam[9]; c.w = w; c.h = h;
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n; i++) {
        double d[3], ta, tb, p[3];
        long ev = 0;
        pixel_ray(&c, px[i], py[i], d);
        out_t[i] = INFINITY;
        if (!ray_aabb(c.eye, d, s->voi_lo, s->voi_hi, &ta, &tb)) continue;
        for (int j = 0; j < 3; j++) p[j] = c.eye[j] + ta * d[j];
        if (field(s, p, NULL) <= 0) { out_t[i] = ta; continue; }
        for (double t = ta; t < tb + dt; t += dt) {
            double t2 = t + dt;
            for (int j = 0; j < 3; j++) p[j] = c.eye[j] + t2 * d[j];
            if (field(s, p, NULL) <= 0) { bisect_root(s, c.eye, d, t, t2, &out_t[i], &ev); break; }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Volumes of interest (Section "Primitive volume of interest"): the
 * primitive's bounding volume offset by the upper end d of its range of
 * interest: sphere (c, r+d), oriented box (c, R, h+d), capsule (a, b, r+d).
 * Ray/volume intervals are analytic. */

static int ray_sphere(const double o[3], const double d[3], const double c[3], double r,
                      double *t0, double *t1) {
    double oc[3] = {o[0] - c[0], o[1] - c[1], o[2] - c[2]};
    double b = oc[0] * d[0] + oc[1] * d[1] + oc[2] * d[2];
    double cc = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2] - r * r;
    double disc = b * b - cc;
    if (disc < 0) return 0;
    double q = sqrt(disc);
    *t0 = -b - q; *t1 = -b + q;
    return 1;
}

static int ray_voi(const or_scene *s, int i, const double o[3], const double d[3], double *t0, double *t1) {
    const double *a = s->par + 16 * i;
    double dd = s->roi[i];
    switch (s->kind[i]) {
    case K_SPHERE:
        return ray_sphere(o, d, a, a[3] + dd, t0, t1);
    case K_BOX:
    case K_TORUS:
    case K_CYLINDER:
    case K_CONE: {
        /* the volume of interest of these three is the oriented box of the
         * primitive's local box grown by d */
        const double *R = s->rot + 9 * i;
        double ext[3] = {a[3], a[4], a[5]};
        if (s->kind[i] != K_BOX) ring_extents(s, i, ext);
        double lo = -INFINITY, hi = INFINITY;
        for (int j = 0; j < 3; j++) {
            double ol = 0, dl = 0;
            for (int q = 0; q < 3; q++) { ol += R[q * 3 + j] * (o[q] - a[q]); dl += R[q * 3 + j] * d[q]; }
            double e = ext[j] + dd;
            if (dl == 0) { if (fabs(ol) > e) return 0; continue; }
            double u = (-e - ol) / dl, v = (e - ol) / dl;
            if (u > v) { double w = u; u = v; v = w; }
            if (u > lo) lo = u;
            if (v < hi) hi = v;
        }
        if (lo > hi) return 0;
        *t0 = lo; *t1 = hi;
        return 1;
    }
    case K_CAPSULE: {
        double r = a[6] + dd, A[3] = {a[0], a[1], a[2]}, B[3] = {a[3], a[4], a[5]};
        double lo = INFINITY, hi = -INFINITY, u, v;
        int any = 0;
        if (ray_sphere(o, d, A, r, &u, &v)) { lo = fmin(lo, u); hi = fmax(hi, v); any = 1; }
        if (ray_sphere(o, d, B, r, &u, &v)) { lo = fmin(lo, u); hi = fmax(hi, v); any = 1; }
        /* cylinder body: |(x - A) x e| <= r and 0 <= (x - A).e <= |B - A| */
        double e[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        double len = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        if (len > 0) {
            for (int j = 0; j < 3; j++) e[j] /= len;
            double oa[3] = {o[0] - A[0], o[1] - A[1], o[2] - A[2]};
            double de = d[0] * e[0] + d[1] * e[1] + d[2] * e[2];
            double oe = oa[0] * e[0] + oa[1] * e[1] + oa[2] * e[2];
            double dp[3], op[3];
            for (int j = 0; j < 3; j++) { dp[j] = d[j] - de * e[j]; op[j] = oa[j] - oe * e[j]; }
            double qa = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
            double qb = op[0] * dp[0] + op[1] * dp[1] + op[2] * dp[2];
            double qc = op[0] * op[0] + op[1] * op[1] + op[2] * op[2] - r * r;
            double c0, c1;
            int ok = 1;
            if (qa > 0) {
                double disc = qb * qb - qa * qc;
                if (disc < 0) ok = 0;
                else { double q = sqrt(disc); c0 = (-qb - q) / qa; c1 = (-qb + q) / qa; }
            } else {
                if (qc > 0) ok = 0; else { c0 = -INFINITY; c1 = INFINITY; }
            }
            if (ok) {
                double s0, s1;
                if (de != 0) {
                    s0 = (0 - oe) / de; s1 = (len - oe) / de;
                    if (s0 > s1) { double w = s0; s0 = s1; s1 = w; }
                } else {
                    if (oe < 0 || oe > len) ok = 0;
                    s0 = -INFINITY; s1 = INFINITY;
                }
                if (ok) {
                    double x0 = fmax(c0, s0), x1 = fmin(c1, s1);
                    if (x0 <= x1) { lo = fmin(lo, x0); hi = fmax(hi, x1); any = 1; }
                }
            }
        }
        if (!any) return 0;
        *t0 = lo; *t1 = hi;
        return 1;
    }
    }
    return 0;
}

/* Brute-force binning reference: for each given pixel and each primitive, the
 * view-depth interval [z_in, z_out] (z = t * (dir . forward)) of the pixel-centre
 * ray inside the primitive's volume of interest, clipped to t >= 0.
 * out_z: n x P x 2 (NaN where the ray misses).  prim_ids: the P primitive
 * node indices in the caller's node numbering. */
void or_voi_intervals(const or_scene *s, const double *cam, int w, int h, const double *px,
                      const double *py, int n, const int32_t *prim_ids, int P, double *out_z) {
    or_camera c; memcpy(c.eye, cam, 3 * sizeof(double)); memcpy(c.target, cam + 3, 3 * sizeof(double));
    memcpy(c.up, cam + 6, 3 * sizeof(double)); c.vfov_deg = cam[9]; c.w = w; c.h = h;
    double fwd[3], right[3], up[3];
    camera_basis(&c, fwd, right, up);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        double d[3];
        pixel_ray(&c, px[i], py[i], d);
        double cs = d[0] * fwd[0] + d[1] * fwd[1] + d[2] * fwd[2];
        for (int q = 0; q < P; q++) {
            double t0, t1;
            double *z = out_z + ((size_t)i * P + q) * 2;
            if (ray_voi(s, prim_ids[q], c.eye, d, &t0, &t1) && t1 >= 0) {
                if (t0 < 0) t0 = 0;
                z[0] = t0 * cs; z[1] = t1 * cs;
            } else {
                z[0] = z[1] = NAN;
            }
        }
    }
}

/* Membership test for the volume of interest of primitive i (pin of
 * "{f_i <= d_i} is inside VOI_i"): returns 1 if x lies in VOI_i. */
int or_in_voi(const or_scene *s, int i, const double x[3]) {
    const double *a = s->par + 16 * i;
    double dd = s->roi[i];
    switch (s->kind[i]) {
    case K_SPHERE: {
        double q = 0; for (int j = 0; j < 3; j++) q += (x[j] - a[j]) * (x[j] - a[j]);
        return sqrt(q) <= a[3] + dd;
    }
    case K_BOX:
    case K_TORUS:
    case K_CYLINDER:
    case K_CONE: {
        const double *R = s->rot + 9 * i;
        double ext[3] = {a[3], a[4], a[5]};
        if (s->kind[i] != K_BOX) ring_extents(s, i, ext);
        for (int j = 0; j < 3; j++) {
            double l = 0; for (int q = 0; q < 3; q++) l += R[q * 3 + j] * (x[q] - a[q]);
            if (fabs(l) > ext[j] + dd) return 0;
        }
        return 1;
    }
    case K_CAPSULE: {
        dual p[3]; for (int j = 0; j < 3; j++) p[j] = dconst(x[j]);
        return prim_dual(s, i, p).v <= dd;
    }
    }
    return 0;
}

/* Primitive field value of node i at x (full precision), for VOI pins. */
double or_prim(const or_scene *s, int i, const double x[3]) {
    dual p[3]; for (int j = 0; j < 3; j++) p[j] = dconst(x[j]);
    return prim_dual(s, i, p).v;
}

/* ------------------------------------------------------------------------ */
/* Step-predictor MLP (not part of the paper): 8 -> 32 -> 32 -> 1 with ReLU,
 * output omega = 1 + (omega_max - 1) * sigmoid(z), loss
 * mean_i w_i (omega_i - target_i)^2 with w_i = over_weight (4 by default) when
 * omega_i > target_i
 * (overshooting costs a rejected step), else 1.
 * Rounding points follow the GPU kernels: inputs and weights arrive already
 * rounded to binary16; the hidden activations are rounded to binary16 before
 * they feed the next layer; in the backward pass the error signals that feed
 * a product are rounded to binary16 as well.  Everything else is FP64.
 * exact != 0 skips those internal roundings (used to pin the backward pass
 * against finite differences of a smooth function).
 * Weight layout: W1[32][8], b1[32], W2[32][32], b2[32], w3[32], b3 (1377). */

/* binary16 round-to-nearest-even of a double, returned as a double. */
double or_round_half(double x) {
    if (isnan(x) || isinf(x) || x == 0) return x;
    double ax = fabs(x);
    if (ax >= 65520.0) return x > 0 ? INFINITY : -INFINITY;
    int e;
    frexp(ax, &e);              /* ax = m * 2^e, m in [0.5, 1) */
    int exp_unb = e - 1;        /* ax in [2^exp_unb, 2^(exp_unb+1)) */
    if (exp_unb < -14) exp_unb = -14;  /* subnormal spacing 2^-24 */
    double ulp = ldexp(1.0, exp_unb - 10);
    double q = ax / ulp;        /* exact: power-of-two scaling */
    double r = nearbyint(q);    /* round-half-even in the default mode */
    double y = r * ulp;
    if (y >= 65520.0) return x > 0 ? INFINITY : -INFINITY;
    return x < 0 ? -y : y;
}

static double relu(double x) { return x > 0 ? x : 0; }

/* Forward and backward over a batch of B samples.
 * X: B x 8 inputs, T: B targets, Wt: 1377 weights (layout above),
 * out_omega: B (may be NULL), out_grad: 1377 (may be NULL).
 * Returns the loss. */
double or_mlp(const double *Wt, const double *X, const double *T, int B, double omega_max,
              int exact, double over_weight, double *out_omega, double *out_grad) {
    const double *W1 = Wt, *b1 = Wt + 256, *W2 = Wt + 288, *b2 = Wt + 1312, *w3 = Wt + 1344,
                 *b3 = Wt + 1376;
    double loss = 0;
    if (out_grad) memset(out_grad, 0, sizeof(double) * 1377);
    for (int s = 0; s < B; s++) {
        const double *x = X + 8 * s;
        double a1[32], h1[32], a2[32], h2[32];
        for (int j = 0; j < 32; j++) {
            double acc = b1[j];
            for (int i = 0; i < 8; i++) acc += W1[j * 8 + i] * x[i];
            a1[j] = acc; h1[j] = exact ? relu(acc) : or_round_half(relu(acc));
        }
        for (int j = 0; j < 32; j++) {
            double acc = b2[j];
            for (int i = 0; i < 32; i++) acc += W2[j * 32 + i] * h1[i];
            a2[j] = acc; h2[j] = exact ? relu(acc) : or_round_half(relu(acc));
        }
        double z = b3[0];
        for (int i = 0; i < 32; i++) z += w3[i] * h2[i];
        double sg = 1.0 / (1.0 + exp(-z));
        double om = 1.0 + (omega_max - 1.0) * sg;
        if (out_omega) out_omega[s] = om;
        double wgt = om > T[s] ? over_weight : 1.0;
        double diff = om - T[s];
        loss += wgt * diff * diff / B;
        if (!out_grad) continue;
        double *gW1 = out_grad, *gb1 = out_grad + 256, *gW2 = out_grad + 288, *gb2 = out_grad + 1312,
               *gw3 = out_grad + 1344, *gb3 = out_grad + 1376;
        double dz = 2.0 * wgt * diff / B * (omega_max - 1.0) * sg * (1.0 - sg);
        gb3[0] += dz;
        double d2[32], d1[32];
        for (int i = 0; i < 32; i++) {
            gw3[i] += dz * h2[i];
            d2[i] = a2[i] > 0 ? dz * w3[i] : 0;
        }
        double d2h[32];
        for (int i = 0; i < 32; i++) d2h[i] = exact ? d2[i] : or_round_half(d2[i]);
        for (int j = 0; j < 32; j++) {
            gb2[j] += d2[j];
            for (int i = 0; i < 32; i++) gW2[j * 32 + i] += d2h[j] * h1[i];
        }
        for (int i = 0; i < 32; i++) {
            double acc = 0;
            for (int j = 0; j < 32; j++) acc += W2[j * 32 + i] * d2h[j];
            d1[i] = a1[i] > 0 ? acc : 0;
        }
        for (int j = 0; j < 32; j++) {
            double dh = exact ? d1[j] : or_round_half(d1[j]);
            gb1[j] += d1[j];
            for (int i = 0; i < 8; i++) gW1[j * 8 + i] += dh * x[i];
        }
    }
    return loss;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
