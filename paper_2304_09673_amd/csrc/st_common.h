// Shared host/device definitions of the synchronized tracer: node bitfield,
// per-node parameter blocks, volume-of-interest records, camera rays.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/st.h"

#define HD __host__ __device__ __forceinline__

namespace st {

// ---------------------------------------------------------------------------
// Node bitfield ("blob", Section 4): isPrimitive(1) nodeop(5) ignoreMod(2)
// isLeft(1) ancestor(23), most significant first.  Nodes are numbered in
// post-order, so the ancestor field holds a node index (the parent here).
constexpr uint32_t kNoNode = 0x7FFFFFu;      // "invalid" 23-bit ancestor
constexpr uint32_t kNoKill = 0xFFFFFFFFu;    // no killing ancestor
// killing ancestors a node's chain row holds (8 words: the first kKillLevels
// killing ancestors, nearest first, padded with kNoKill, then their count)
constexpr int kKillLevels = 7;
constexpr int kMaxDepth = 31;                // evaluation stack bound
constexpr int kStack = 32;

HD uint32_t blob_pack(bool prim, uint32_t op, uint32_t ignore, bool is_left, uint32_t anc) {
    return (uint32_t(prim) << 31) | ((op & 31u) << 26) | ((ignore & 3u) << 24) |
           (uint32_t(is_left) << 23) | (anc & 0x7FFFFFu);
}
HD bool blob_prim(uint32_t b) { return (b >> 31) != 0; }
HD uint32_t blob_op(uint32_t b) { return (b >> 26) & 31u; }
HD uint32_t blob_ignore(uint32_t b) { return (b >> 24) & 3u; }
HD bool blob_left(uint32_t b) { return ((b >> 23) & 1u) != 0; }
HD uint32_t blob_anc(uint32_t b) { return b & 0x7FFFFFu; }

// ignoreMod values (Section 9): behaviour of an operator when one operand is
// absent from the pruned tree.  Bit 0: ignore (return +inf) when the right
// operand is absent; bit 1: when the left operand is absent.
constexpr uint32_t kIgnoreNever = 0u;   // union-like
constexpr uint32_t kIgnoreLeftAbsent = 2u;   // difference-like
constexpr uint32_t kIgnoreAny = 3u;     // intersection-like

HD bool is_prim_kind(uint32_t k) { return k <= ST_CONE; }
// node class of the evaluation counters: sphere, primitive in a rotated box
// frame (box, torus, cylinder, cone), capsule, operator
HD uint32_t node_class(uint32_t k) { return k == ST_SPHERE ? 0u : k == ST_CAPSULE ? 2u : k <= ST_CONE ? 1u : 3u; }
// counts[node_class(k)] += 1 with constant indices only (a run-time index
// into a small per-lane array would place it in scratch memory)
HD void count_class(uint32_t (&counts)[4], uint32_t k) {
    const uint32_t c = node_class(k);
    counts[0] += c == 0u ? 1u : 0u;
    counts[1] += c == 1u ? 1u : 0u;
    counts[2] += c == 2u ? 1u : 0u;
    counts[3] += c == 3u ? 1u : 0u;
}
HD bool is_op_kind(uint32_t k) { return k >= ST_UNION && k <= ST_SDIFF; }
HD bool is_compact_kind(uint32_t k) { return k >= ST_SUNION && k <= ST_SDIFF; }
HD uint32_t ignore_of(uint32_t k) {
    return (k == ST_INTER || k == ST_SINTER) ? kIgnoreAny
         : (k == ST_DIFF || k == ST_SDIFF) ? kIgnoreLeftAbsent : kIgnoreNever;
}

// View entries: node index (24 bits) | node kind << 24.
constexpr uint32_t kMaxNodes = 1u << 23;
HD uint32_t ventry(uint32_t node, uint32_t kind) { return node | (kind << 24); }
HD uint32_t ventry_node(uint32_t e) { return e & 0xFFFFFFu; }
HD uint32_t ventry_kind(uint32_t e) { return e >> 24; }

// ---------------------------------------------------------------------------
// Per-node parameter block: 16 floats (64 B), read with uniform addresses.
//  sphere : [0..2] c, [3] r
//  box    : [0..2] c, [4..6] axis 0, [7] h0, [8..10] axis 1, [11] h1,
//           [12..14] axis 2, [15] h2  (local coordinate i = axis_i . (p-c))
//  capsule: [0..2] a, [3] r, [4..6] b - a, [7] 1/|b-a|^2 (0 when a = b)
//  torus  : [0..2] c, [3] R, [4..6] axis 0, [7] r, [8..10] axis 1 (of
//           revolution), [12..14] axis 2
//  cylinder: [0..2] c, [3] radius, [4..6] axis 0, [7] half height, [8..10]
//           axis 1 (the cylinder's axis), [12..14] axis 2
//  operator: [0] k, [1] 1/k, [2] s = 6k/(6 d_o - k), [3] d_o,
//            [4] Lipschitz factor 1 + k/(6 d_o - k) (1 for sharp),
//            [5] k/6
struct NodePar { float v[16]; };

// Per-primitive volume of interest (Section 6.1): the primitive's bounding
// volume offset by its range of interest d.
//  [0..2] bounding-sphere centre, [3] bounding-sphere radius,
//  sphere : [4..6] c, [7] r + d
//  box    : [4..6] c, [8..10] axis0, [11] h0+d, [12..14] axis1, [15] h1+d,
//           [16..18] axis2, [19] h2+d
//  capsule: [4..6] a, [7] r + d, [8..10] b
//  (a torus or cylinder has the oriented-box volume of its local box grown
//  by d, stored as a box)
//  [20] kind, [21] node index (as float bits)
struct Voi { float v[24]; };

// ---------------------------------------------------------------------------
// Camera and pixel rays, shared by the A-buffer build and the tracer so that
// both see bitwise identical rays (explicit fma, no contraction freedom).
struct DevCam {
    float eye[3], fwd[3], right[3], up[3];
    float tx, ty;          // tan(fov/2) * W/H, tan(fov/2)
    float inv_w2, inv_h2;  // 2/W, 2/H
    int32_t w, h;
};

struct Ray { float o[3], d[3], cosv; };

HD Ray pixel_ray(const DevCam& c, int i, int j) {
    float x = fmaf(float(i) + 0.5f, c.inv_w2, -1.0f) * c.tx;
    float y = fmaf(-(float(j) + 0.5f), c.inv_h2, 1.0f) * c.ty;
    float d0 = fmaf(x, c.right[0], fmaf(y, c.up[0], c.fwd[0]));
    float d1 = fmaf(x, c.right[1], fmaf(y, c.up[1], c.fwd[1]));
    float d2 = fmaf(x, c.right[2], fmaf(y, c.up[2], c.fwd[2]));
    float l2 = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
    float inv = 1.0f / sqrtf(l2);
    Ray r;
    r.o[0] = c.eye[0]; r.o[1] = c.eye[1]; r.o[2] = c.eye[2];
    r.d[0] = d0 * inv; r.d[1] = d1 * inv; r.d[2] = d2 * inv;
    r.cosv = fmaf(r.d[0], c.fwd[0], fmaf(r.d[1], c.fwd[1], r.d[2] * c.fwd[2]));
    return r;
}

}  // namespace st
