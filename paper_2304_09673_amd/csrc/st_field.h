// Device evaluation of blobtree nodes in FP32, as values (float) or as
// values with their spatial gradient (Dual, forward-mode differentiation).
//
// Primitives are exact signed distances (Section 6.1 asks for Lipschitz <= 1).
// Operators (Section 5): sharp CSG; the C2 polynomial blends
//   g_union(a,b,K) = min(a,b) - disp(a,b,K), g_inter = max + disp,
//   g_diff(a,b,K) = max(a,-b) + disp(a,-b,K),
//   disp(a,b,K) = K/6 max(1 - |a-b|/K, 0)^3;
// and the compact operators G: when both operands are <= d_o the blend radius
// is interpolated from the first blend value x = g(a,b,k) by
//   b_r(x) = k max(1 - 6x/(6 d_o - k), 0) = max(k - s x, 0),  s = 6k/(6 d_o - k),
// (upper-clamped to k for intersection and difference, applied to |x| for
// the difference) and G = g(a,b,b_r); otherwise G is the sharp operator.
// A zero blend radius gives zero displacement (the text's NaN filter).
#pragma once

#include "st_common.h"

namespace st {

struct Dual {
    float v, gx, gy, gz;
};

// Node parameters are read through the constant address space: the addresses
// are wave-uniform and the data is read-only while tracing, so the loads
// become scalar loads into SGPRs instead of per-lane vector copies.
typedef __attribute__((address_space(4))) const float cfloat;

// ---- scalar helpers, overloaded for float and Dual ---------------------------
__device__ __forceinline__ float val(float a) { return a; }
__device__ __forceinline__ float val(const Dual& a) { return a.v; }

__device__ __forceinline__ float mk(float v, float) { return v; }

__device__ __forceinline__ Dual operator+(const Dual& a, const Dual& b) { return {a.v + b.v, a.gx + b.gx, a.gy + b.gy, a.gz + b.gz}; }
__device__ __forceinline__ Dual operator-(const Dual& a, const Dual& b) { return {a.v - b.v, a.gx - b.gx, a.gy - b.gy, a.gz - b.gz}; }
__device__ __forceinline__ Dual operator-(const Dual& a) { return {-a.v, -a.gx, -a.gy, -a.gz}; }
__device__ __forceinline__ Dual operator*(const Dual& a, float s) { return {a.v * s, a.gx * s, a.gy * s, a.gz * s}; }
__device__ __forceinline__ Dual operator*(const Dual& a, const Dual& b) {
    return {a.v * b.v, a.gx * b.v + a.v * b.gx, a.gy * b.v + a.v * b.gy, a.gz * b.v + a.v * b.gz};
}
__device__ __forceinline__ Dual operator+(const Dual& a, float s) { return {a.v + s, a.gx, a.gy, a.gz}; }
__device__ __forceinline__ Dual operator-(const Dual& a, float s) { return {a.v - s, a.gx, a.gy, a.gz}; }
__device__ __forceinline__ Dual operator-(float s, const Dual& a) { return {s - a.v, -a.gx, -a.gy, -a.gz}; }

__device__ __forceinline__ float cst(float c, float) { return c; }
__device__ __forceinline__ Dual cst(float c, const Dual&) { return {c, 0.f, 0.f, 0.f}; }

__device__ __forceinline__ float fmin_(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ Dual fmin_(const Dual& a, const Dual& b) { return b.v < a.v ? b : a; }
__device__ __forceinline__ float fmax_(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ Dual fmax_(const Dual& a, const Dual& b) { return b.v > a.v ? b : a; }
__device__ __forceinline__ float fabs_(float a) { return fabsf(a); }
__device__ __forceinline__ Dual fabs_(const Dual& a) { return a.v < 0.f ? -a : a; }
__device__ __forceinline__ float relu_(float a) { return fmaxf(a, 0.f); }
__device__ __forceinline__ Dual relu_(const Dual& a) { return a.v > 0.f ? a : Dual{0.f, 0.f, 0.f, 0.f}; }
// hardware square root and reciprocal (1 ulp), not the correctly rounded
// library sequences: the parity tolerances are orders of magnitude looser
__device__ __forceinline__ float sqrt_(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ Dual sqrt_(const Dual& a) {
    float r = __builtin_amdgcn_sqrtf(a.v);
    float h = r > 0.f ? 0.5f * __builtin_amdgcn_rcpf(r) : 0.f;
    return {r, a.gx * h, a.gy * h, a.gz * h};
}
__device__ __forceinline__ float rcp_(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ Dual rcp_(const Dual& a) {
    float r = __builtin_amdgcn_rcpf(a.v);
    float m = -r * r;
    return {r, a.gx * m, a.gy * m, a.gz * m};
}
__device__ __forceinline__ float clamp01_(float a) { return fminf(fmaxf(a, 0.f), 1.f); }
__device__ __forceinline__ Dual clamp01_(const Dual& a) {
    if (a.v <= 0.f) return {0.f, 0.f, 0.f, 0.f};
    if (a.v >= 1.f) return {1.f, 0.f, 0.f, 0.f};
    return a;
}

// Point: coordinates as value or as dual (gradient seeds e_x, e_y, e_z).
template <class T> struct P3 { T x, y, z; };
__device__ __forceinline__ P3<float> make_point(float x, float y, float z, float) { return {x, y, z}; }
__device__ __forceinline__ P3<Dual> make_point(float x, float y, float z, const Dual&) {
    return {{x, 1.f, 0.f, 0.f}, {y, 0.f, 1.f, 0.f}, {z, 0.f, 0.f, 1.f}};
}

// ---- primitives -----------------------------------------------------------
template <class T>
__device__ __forceinline__ T prim_sphere(const cfloat* q, const P3<T>& p) {
    T dx = p.x - q[0], dy = p.y - q[1], dz = p.z - q[2];
    return sqrt_(dx * dx + dy * dy + dz * dz) - q[3];
}

template <class T>
__device__ __forceinline__ T prim_box(const cfloat* q, const P3<T>& p) {
    T dx = p.x - q[0], dy = p.y - q[1], dz = p.z - q[2];
    T l0 = fabs_(dx * q[4] + dy * q[5] + dz * q[6]) - q[7];
    T l1 = fabs_(dx * q[8] + dy * q[9] + dz * q[10]) - q[11];
    T l2 = fabs_(dx * q[12] + dy * q[13] + dz * q[14]) - q[15];
    T o0 = relu_(l0), o1 = relu_(l1), o2 = relu_(l2);
    T outside = sqrt_(o0 * o0 + o1 * o1 + o2 * o2);
    T inside = fmin_(fmax_(fmax_(l0, l1), l2), cst(0.f, l0));
    return outside + inside;
}

template <class T>
__device__ __forceinline__ T prim_capsule(const cfloat* q, const P3<T>& p) {
    T ax = p.x - q[0], ay = p.y - q[1], az = p.z - q[2];
    T h = clamp01_((ax * q[4] + ay * q[5] + az * q[6]) * q[7]);
    T wx = ax - h * q[4], wy = ay - h * q[5], wz = az - h * q[6];
    return sqrt_(wx * wx + wy * wy + wz * wz) - q[3];
}

// ---- operators ------------------------------------------------------------
// displacement K/6 max(1 - |a-b|/K, 0)^3 given |a-b| (K > 0 checked by caller)
template <class T>
__device__ __forceinline__ T disp_(const T& diff, const T& K) {
    T h = relu_(cst(1.f, diff) - diff * rcp_(K));
    return K * (h * h * h) * (1.0f / 6.0f);
}

template <class T>
__device__ __forceinline__ T op_eval(uint32_t kind, const cfloat* q, const T& a, const T& b, uint32_t& sm) {
    switch (kind) {
    case ST_UNION: return fmin_(a, b);
    case ST_INTER: return fmax_(a, b);
    case ST_DIFF: return fmax_(a, -b);
    case ST_SUNION: {
        T m = fmin_(a, b);
        if (val(a) <= q[3] && val(b) <= q[3]) {
            T diff = fabs_(a - b);
            T h = relu_(cst(1.f, a) - diff * q[1]);
            T x = m - (h * h * h) * q[5];                 // g_union(a, b, k)
            T K = relu_(cst(q[0], a) - x * q[2]);         // b_r(x), unclamped
            if (val(K) > 0.f) m = m - disp_(diff, K);
            sm++;
        }
        return m;
    }
    case ST_SINTER: {
        T m = fmax_(a, b);
        if (val(a) <= q[3] && val(b) <= q[3]) {
            T diff = fabs_(a - b);
            T h = relu_(cst(1.f, a) - diff * q[1]);
            T x = m + (h * h * h) * q[5];                 // g_inter(a, b, k)
            T K = fmin_(relu_(cst(q[0], a) - x * q[2]), cst(q[0], a));
            if (val(K) > 0.f) m = m + disp_(diff, K);
            sm++;
        }
        return m;
    }
    case ST_SDIFF: {
        T nb = -b;
        T m = fmax_(a, nb);
        if (val(a) <= q[3] && val(b) <= q[3]) {
            T diff = fabs_(a - nb);
            T h = relu_(cst(1.f, a) - diff * q[1]);
            T x = m + (h * h * h) * q[5];                 // g_diff(a, b, k)
            T K = fmin_(relu_(cst(q[0], a) - fabs_(x) * q[2]), cst(q[0], a));
            if (val(K) > 0.f) m = m + disp_(diff, K);
            sm++;
        }
        return m;
    }
    }
    return cst(__builtin_inff(), a);
}

// torus and capped cylinder: exact distances in the local frame, whose
// y axis is the axis of revolution; rad = distance to that axis.
//  torus:    |(rad - R, ly)| - r
//  cylinder: w = (rad - radius, |ly| - h): |max(w, 0)| + min(max(wx, wy), 0)
template <class T>
__device__ __forceinline__ T prim_torus(const cfloat* q, const P3<T>& p) {
    T dx = p.x - q[0], dy = p.y - q[1], dz = p.z - q[2];
    T lx = dx * q[4] + dy * q[5] + dz * q[6];
    T ly = dx * q[8] + dy * q[9] + dz * q[10];
    T lz = dx * q[12] + dy * q[13] + dz * q[14];
    T qx = sqrt_(lx * lx + lz * lz) - q[3];
    return sqrt_(qx * qx + ly * ly) - q[7];
}

template <class T>
__device__ __forceinline__ T prim_cylinder(const cfloat* q, const P3<T>& p) {
    T dx = p.x - q[0], dy = p.y - q[1], dz = p.z - q[2];
    T lx = dx * q[4] + dy * q[5] + dz * q[6];
    T ly = dx * q[8] + dy * q[9] + dz * q[10];
    T lz = dx * q[12] + dy * q[13] + dz * q[14];
    T wx = sqrt_(lx * lx + lz * lz) - q[3];
    T wy = fabs_(ly) - q[7];
    T ox = relu_(wx), oy = relu_(wy);
    return sqrt_(ox * ox + oy * oy) + fmin_(fmax_(wx, wy), cst(0.f, wx));
}

// Capped cone, axis local y: radius q[3] at y = -q[7], q[11] at y = +q[7];
// q[15] = 1 / |(q[11] - q[3], 2 q[7])|.  In the meridian half-plane (rho, y)
// the solid is a trapezoid.  Inside it the distance is that to the nearer
// face line (the section through the axis is convex); outside, the smaller
// of the distances to the cap segment on the point's side and to the side
// segment, the latter as the distance to the side's line when the foot
// falls inside the segment, and the former as the distance to the cap's
// plane above the disk (linear forms whose gradients stay exact at the
// surface, where a square root of a near-zero or zero square would not).
template <class T>
__device__ __forceinline__ T prim_cone(const cfloat* q, const P3<T>& p) {
    T dx = p.x - q[0], dy = p.y - q[1], dz = p.z - q[2];
    T lx = dx * q[4] + dy * q[5] + dz * q[6];
    T ly = dx * q[8] + dy * q[9] + dz * q[10];
    T lz = dx * q[12] + dy * q[13] + dz * q[14];
    const float rb = q[3], h = q[7], rt = q[11], il = q[15];
    const float ex = rt - rb, ey = 2.f * h;
    T rho = sqrt_(lx * lx + lz * lz);
    T px = rho - rb, py = ly + h;        // relative to the side's bottom end
    T sd = (px * ey - py * ex) * il;     // signed distance to the side's line, > 0 outside
    T cy = fabs_(ly) - h;                // signed distance to the nearer cap's plane
    if (val(sd) < 0.f && val(cy) < 0.f) return fmax_(sd, cy);
    const float rcap = val(ly) < 0.f ? rb : rt;
    // the cap segment: its plane when the point is above the disk (a hit
    // point can lie exactly on that plane, where the square root of 0 would
    // give a zero gradient), else its rim
    T cx = relu_(rho - rcap);
    T dcap = val(cx) > 0.f ? sqrt_(cx * cx + cy * cy) : fabs_(cy);
    T t = (px * ex + py * ey) * (il * il);   // foot on the side, 0 at the bottom end, 1 at the top
    T dside;
    if (val(t) > 0.f && val(t) < 1.f) {
        dside = fabs_(sd);
    } else {
        const float te = val(t) <= 0.f ? 0.f : 1.f;
        T bx = px - te * ex, by = py - te * ey;
        dside = sqrt_(bx * bx + by * by);
    }
    return fmin_(dcap, dside);
}

template <class T>
__device__ __forceinline__ T prim_eval(uint32_t kind, const cfloat* q, const P3<T>& p) {
    if (kind == ST_SPHERE) return prim_sphere(q, p);
    if (kind == ST_BOX) return prim_box(q, p);
    if (kind == ST_CAPSULE) return prim_capsule(q, p);
    if (kind == ST_TORUS) return prim_torus(q, p);
    if (kind == ST_CONE) return prim_cone(q, p);
    return prim_cylinder(q, p);
}

}  // namespace st
