// Interval of a pixel ray inside a primitive's volume of interest (Section
// 6.1: the primitive's bounding volume offset by its range of interest),
// shared by the tile A-buffer test and the per-pixel dexel build.
#pragma once

#include "st_common.h"

namespace st {

// ray / volume-of-interest interval along the unit ray (t), false on a miss
__device__ __forceinline__ bool ray_sphere(const float o[3], const float d[3], float cx, float cy, float cz,
                                           float R, float& t0, float& t1) {
    float ox = o[0] - cx, oy = o[1] - cy, oz = o[2] - cz;
    float b = ox * d[0] + oy * d[1] + oz * d[2];
    // distance of the centre to the ray, computed without cancellation
    float qx = ox - b * d[0], qy = oy - b * d[1], qz = oz - b * d[2];
    float disc = R * R - (qx * qx + qy * qy + qz * qz);
    if (disc < 0.f) return false;
    float s = sqrtf(disc);
    t0 = -b - s;
    t1 = -b + s;
    return true;
}

__device__ __forceinline__ bool ray_voi(const Voi& v, const float o[3], const float d[3], float& t0, float& t1) {
    int kind = int(v.v[20]);
    if (kind == ST_SPHERE) return ray_sphere(o, d, v.v[4], v.v[5], v.v[6], v.v[7], t0, t1);
    if (kind == ST_BOX) {
        float rx = o[0] - v.v[4], ry = o[1] - v.v[5], rz = o[2] - v.v[6];
        float lo = -__builtin_inff(), hi = __builtin_inff();
        for (int a = 0; a < 3; a++) {
            const float* ax = v.v + 8 + 4 * a;
            float ol = ax[0] * rx + ax[1] * ry + ax[2] * rz;
            float dl = ax[0] * d[0] + ax[1] * d[1] + ax[2] * d[2];
            float e = ax[3];
            if (fabsf(dl) < 1e-20f) {
                if (fabsf(ol) > e) return false;
                continue;
            }
            float inv = 1.0f / dl;
            float u = (-e - ol) * inv, w = (e - ol) * inv;
            lo = fmaxf(lo, fminf(u, w));
            hi = fminf(hi, fmaxf(u, w));
        }
        if (lo > hi) return false;
        t0 = lo; t1 = hi;
        return true;
    }
    // capsule: end spheres and the cylinder between the end planes
    float R = v.v[7];
    float ax = v.v[4], ay = v.v[5], az = v.v[6], bx = v.v[8], by = v.v[9], bz = v.v[10];
    float lo = __builtin_inff(), hi = -__builtin_inff();
    float u, w;
    if (ray_sphere(o, d, ax, ay, az, R, u, w)) { lo = fminf(lo, u); hi = fmaxf(hi, w); }
    if (ray_sphere(o, d, bx, by, bz, R, u, w)) { lo = fminf(lo, u); hi = fmaxf(hi, w); }
    float ex = bx - ax, ey = by - ay, ez = bz - az;
    float len = sqrtf(ex * ex + ey * ey + ez * ez);
    if (len > 0.f) {
        float il = 1.0f / len;
        ex *= il; ey *= il; ez *= il;
        float oax = o[0] - ax, oay = o[1] - ay, oaz = o[2] - az;
        float de = d[0] * ex + d[1] * ey + d[2] * ez;
        float oe = oax * ex + oay * ey + oaz * ez;
        float dpx = d[0] - de * ex, dpy = d[1] - de * ey, dpz = d[2] - de * ez;
        float opx = oax - oe * ex, opy = oay - oe * ey, opz = oaz - oe * ez;
        float qa = dpx * dpx + dpy * dpy + dpz * dpz;
        float qb = opx * dpx + opy * dpy + opz * dpz;
        float qc = opx * opx + opy * opy + opz * opz - R * R;
        if (qa > 1e-20f) {
            // distance of closest approach to the axis line, cancellation free
            float tc = -qb / qa;
            float cx = opx + tc * dpx, cy = opy + tc * dpy, cz = opz + tc * dpz;
            float disc = (R * R - (cx * cx + cy * cy + cz * cz)) / qa;
            if (disc >= 0.f) {
                float sq = sqrtf(disc);
                float c0 = tc - sq, c1 = tc + sq;
                float s0, s1;
                if (fabsf(de) > 1e-20f) {
                    float ide = 1.0f / de;
                    s0 = -oe * ide; s1 = (len - oe) * ide;
                    if (s0 > s1) { float tmp = s0; s0 = s1; s1 = tmp; }
                } else {
                    if (oe < 0.f || oe > len) { s0 = 1.f; s1 = 0.f; } else { s0 = -__builtin_inff(); s1 = __builtin_inff(); }
                }
                float x0 = fmaxf(c0, s0), x1 = fminf(c1, s1);
                if (x0 <= x1) { lo = fminf(lo, x0); hi = fmaxf(hi, x1); }
            }
        } else if (qc <= 0.f) {
            float s0, s1;
            if (fabsf(de) > 1e-20f) {
                float ide = 1.0f / de;
                s0 = -oe * ide; s1 = (len - oe) * ide;
                if (s0 > s1) { float tmp = s0; s0 = s1; s1 = tmp; }
                lo = fminf(lo, s0); hi = fmaxf(hi, s1);
            }
        }
    }
    if (!(lo <= hi)) return false;
    t0 = lo; t1 = hi;
    return true;
}

}  // namespace st
