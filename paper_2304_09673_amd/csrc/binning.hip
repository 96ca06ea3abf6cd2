// Tile A-buffer of volumes of interest (Section 6 of Zanni 2023).
//
// The paper rasterises every volume of interest at tile resolution: a
// geometry shader emits an impostor, its fragment shader intersects the
// tile's 8x8 rays with the volume, keeps the minimum entry and maximum exit
// depth, and inserts {primitive, z_in, z_out} into the tile's linked list kept
// sorted by entry depth (Section 6.2).  Here the same per-tile lists are built
// with data-parallel kernels, tile-major:
//   voi      : per primitive, the volume of interest (bound offset by the
//              range of interest) and a bounding sphere;
//   rect     : per primitive, the conservative screen rectangle of tiles its
//              bounding sphere can touch (exact tangent planes of a sphere);
//   count    : per tile, the number of primitives whose rectangle covers it;
//   scan     : tile segments (CSR) of candidate slots;
//   scatter  : every primitive's index written to a slot of each tile of its
//              rectangle;
//   test     : per tile, the tile's pixel-centre rays (computed once, held in
//              registers) are intersected with each candidate's volume; the
//              minimum entry / maximum exit view depth of the rays that hit
//              is written in the slot (a miss writes an empty interval);
//   prune    : per tile, misses are dropped, and so are the entries whose
//              primitive cannot reach the root for any subset of the tile's
//              list (not in the paper; see tile_prune below); the kept ones
//              are compacted to the front of the segment;
//   sort     : per tile, entries sorted by (z_in, primitive) in LDS (bitonic),
//              and the tile's largest depth overlap of intervals computed.
#include <algorithm>

#include "st_internal.h"
#include "st_prune.h"
#include "st_voi.h"

namespace st {

// ---------------------------------------------------------------------------
// volumes of interest
__global__ void voi_kernel(const uint32_t* __restrict__ prims, int P, const NodePar* __restrict__ par,
                           const float* __restrict__ roi, const uint32_t* __restrict__ blob,
                           Voi* __restrict__ out) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    uint32_t node = prims[p];
    const float* q = par[node].v;
    float d = roi[node];
    uint32_t kind = blob_op(blob[node]);
    Voi v;
    for (int j = 0; j < 24; j++) v.v[j] = 0.f;
    if (kind == ST_SPHERE) {
        float R = q[3] + d;
        v.v[0] = q[0]; v.v[1] = q[1]; v.v[2] = q[2]; v.v[3] = R;
        v.v[4] = q[0]; v.v[5] = q[1]; v.v[6] = q[2]; v.v[7] = R;
    } else if (kind == ST_BOX || kind == ST_TORUS || kind == ST_CYLINDER || kind == ST_CONE) {
        // oriented box of the local box grown by d (torus: ring radius R,
        // tube r; cylinder: radius, half height along axis 1; cone: the
        // larger end radius, half height)
        float e0, e1, e2;
        if (kind == ST_BOX) {
            e0 = q[7] + d; e1 = q[11] + d; e2 = q[15] + d;
        } else if (kind == ST_TORUS) {
            e0 = q[3] + q[7] + d; e1 = q[7] + d; e2 = e0;
        } else if (kind == ST_CONE) {
            e0 = fmaxf(q[3], q[11]) + d; e1 = q[7] + d; e2 = e0;
        } else {
            e0 = q[3] + d; e1 = q[7] + d; e2 = e0;
        }
        kind = ST_BOX;
        v.v[0] = q[0]; v.v[1] = q[1]; v.v[2] = q[2];
        v.v[3] = sqrtf(e0 * e0 + e1 * e1 + e2 * e2) * 1.0001f;
        v.v[4] = q[0]; v.v[5] = q[1]; v.v[6] = q[2];
        for (int a = 0; a < 3; a++) {
            for (int c = 0; c < 3; c++) v.v[8 + 4 * a + c] = q[4 + 4 * a + c];
        }
        v.v[11] = e0; v.v[15] = e1; v.v[19] = e2;
    } else {
        float R = q[3] + d;
        float bx = q[0] + q[4], by = q[1] + q[5], bz = q[2] + q[6];
        float hl = 0.5f * sqrtf(q[4] * q[4] + q[5] * q[5] + q[6] * q[6]);
        v.v[0] = 0.5f * (q[0] + bx); v.v[1] = 0.5f * (q[1] + by); v.v[2] = 0.5f * (q[2] + bz);
        v.v[3] = (hl + R) * 1.0001f;
        v.v[4] = q[0]; v.v[5] = q[1]; v.v[6] = q[2]; v.v[7] = R;
        v.v[8] = bx; v.v[9] = by; v.v[10] = bz;
    }
    v.v[20] = float(kind);
    v.v[21] = __uint_as_float(node);
    out[p] = v;
}

// ---------------------------------------------------------------------------
// screen rectangle of tiles touched by a bounding sphere
__device__ __forceinline__ void slope_range(float c, float z, float r, float& lo, float& hi) {
    // tangent lines through the eye to the circle (c, z) of radius r: slope c/z
    float den = z * z - r * r;
    float sq = r * sqrtf(fmaxf(c * c + den, 0.f));
    lo = (c * z - sq) / den;
    hi = (c * z + sq) / den;
}

// Conservative pixel rectangle [i0, i1] x [j0, j1] (clamped to the image) of
// the pixel-centre rays that can meet a bounding sphere: exact tangent lines
// through the eye, one pixel of margin; the whole image when the sphere
// reaches the eye plane; false when it lies behind the eye or off screen.
__device__ __forceinline__ bool sphere_pixels(float sx, float sy, float sz, float radius, const DevCam& cam, int& i0,
                                              int& i1, int& j0, int& j1) {
    float rx = sx - cam.eye[0], ry = sy - cam.eye[1], rz = sz - cam.eye[2];
    float cx = rx * cam.right[0] + ry * cam.right[1] + rz * cam.right[2];
    float cy = rx * cam.up[0] + ry * cam.up[1] + rz * cam.up[2];
    float cz = rx * cam.fwd[0] + ry * cam.fwd[1] + rz * cam.fwd[2];
    float r = radius * 1.001f + 1e-5f;
    i0 = 0; i1 = cam.w - 1; j0 = 0; j1 = cam.h - 1;
    if (cz + r <= 0.f) return false;   // entirely behind the eye
    if (cz > r * 1.01f + 1e-4f) {
        float xl, xh, yl, yh;
        slope_range(cx, cz, r, xl, xh);
        slope_range(cy, cz, r, yl, yh);
        // pixel centre coordinate u = i + 1/2 = (x/tx + 1) W/2;  v = j + 1/2 = (1 - y/ty) H/2
        float ul = (xl / cam.tx + 1.f) * 0.5f * cam.w, uh = (xh / cam.tx + 1.f) * 0.5f * cam.w;
        float vl = (1.f - yh / cam.ty) * 0.5f * cam.h, vh = (1.f - yl / cam.ty) * 0.5f * cam.h;
        i0 = max(i0, int(floorf(ul - 0.5f)) - 1);
        i1 = min(i1, int(ceilf(uh - 0.5f)) + 1);
        j0 = max(j0, int(floorf(vl - 0.5f)) - 1);
        j1 = min(j1, int(ceilf(vh - 0.5f)) + 1);
    }
    return i0 <= i1 && j0 <= j1;
}

// Conservative pixel rectangle of a volume of interest, tighter than that of
// its bounding sphere: a capsule lies in the convex hull of its two end
// spheres, whose projection is bounded by the union of the two spheres'
// rectangles; a box projects into the hull of its eight projected corners
// when they all lie in front of the eye (one pixel of margin, as for the
// spheres).  Other cases use the bounding sphere.
__device__ __forceinline__ bool voi_pixels(const Voi& v, const DevCam& cam, int& i0, int& i1, int& j0, int& j1) {
    const int kind = int(v.v[20]);
    if (kind == ST_CAPSULE) {
        int a0, a1, b0, b1, c0, c1, d0, d1;
        const bool ha = sphere_pixels(v.v[4], v.v[5], v.v[6], v.v[7], cam, a0, a1, b0, b1);
        const bool hb = sphere_pixels(v.v[8], v.v[9], v.v[10], v.v[7], cam, c0, c1, d0, d1);
        if (!ha && !hb) return false;
        i0 = ha ? (hb ? min(a0, c0) : a0) : c0;
        i1 = ha ? (hb ? max(a1, c1) : a1) : c1;
        j0 = ha ? (hb ? min(b0, d0) : b0) : d0;
        j1 = ha ? (hb ? max(b1, d1) : b1) : d1;
        return true;
    }
    if (kind == ST_BOX) {
        float umin = __builtin_inff(), umax = -__builtin_inff(), vmin = __builtin_inff(), vmax = -__builtin_inff();
        bool front = true;
        for (int c = 0; c < 8; c++) {
            float p[3];
            for (int k = 0; k < 3; k++) {
                p[k] = v.v[4 + k] - cam.eye[k];
                for (int a = 0; a < 3; a++) p[k] += ((c >> a) & 1 ? 1.f : -1.f) * v.v[8 + 4 * a + 3] * v.v[8 + 4 * a + k];
            }
            const float x = p[0] * cam.right[0] + p[1] * cam.right[1] + p[2] * cam.right[2];
            const float y = p[0] * cam.up[0] + p[1] * cam.up[1] + p[2] * cam.up[2];
            const float z = p[0] * cam.fwd[0] + p[1] * cam.fwd[1] + p[2] * cam.fwd[2];
            front = front && z > 1e-3f;
            const float u = (x / (z * cam.tx) + 1.f) * 0.5f * cam.w, w = (1.f - y / (z * cam.ty)) * 0.5f * cam.h;
            umin = fminf(umin, u); umax = fmaxf(umax, u); vmin = fminf(vmin, w); vmax = fmaxf(vmax, w);
        }
        if (front) {
            // corner extent with a relative margin for FP32 rounding of the projection
            const float mu = 1e-4f * (fabsf(umin) + fabsf(umax)) + 1e-3f, mv = 1e-4f * (fabsf(vmin) + fabsf(vmax)) + 1e-3f;
            i0 = max(0, int(floorf(umin - mu - 0.5f)) - 1);
            i1 = min(cam.w - 1, int(ceilf(umax + mu - 0.5f)) + 1);
            j0 = max(0, int(floorf(vmin - mv - 0.5f)) - 1);
            j1 = min(cam.h - 1, int(ceilf(vmax + mv - 0.5f)) + 1);
            return i0 <= i1 && j0 <= j1;
        }
    }
    return sphere_pixels(v.v[0], v.v[1], v.v[2], v.v[3], cam, i0, i1, j0, j1);
}

// Conservative pixel rectangle of an axis-aligned box (lo, hi): its eight
// corners projected when they all lie in front of the eye (a relative margin
// and one pixel, as for the boxes above), else its bounding sphere.
__device__ __forceinline__ bool aabb_pixels(const float* lo, const float* hi, const DevCam& cam, int& i0, int& i1,
                                            int& j0, int& j1) {
    float umin = __builtin_inff(), umax = -__builtin_inff(), vmin = __builtin_inff(), vmax = -__builtin_inff();
    bool front = true;
    for (int c = 0; c < 8; c++) {
        const float px = ((c & 1) ? hi[0] : lo[0]) - cam.eye[0];
        const float py = ((c & 2) ? hi[1] : lo[1]) - cam.eye[1];
        const float pz = ((c & 4) ? hi[2] : lo[2]) - cam.eye[2];
        const float x = px * cam.right[0] + py * cam.right[1] + pz * cam.right[2];
        const float y = px * cam.up[0] + py * cam.up[1] + pz * cam.up[2];
        const float z = px * cam.fwd[0] + py * cam.fwd[1] + pz * cam.fwd[2];
        front = front && z > 1e-3f;
        const float u = (x / (z * cam.tx) + 1.f) * 0.5f * cam.w, w = (1.f - y / (z * cam.ty)) * 0.5f * cam.h;
        umin = fminf(umin, u); umax = fmaxf(umax, u); vmin = fminf(vmin, w); vmax = fmaxf(vmax, w);
    }
    if (front) {
        const float mu = 1e-4f * (fabsf(umin) + fabsf(umax)) + 1e-3f, mv = 1e-4f * (fabsf(vmin) + fabsf(vmax)) + 1e-3f;
        i0 = max(0, int(floorf(umin - mu - 0.5f)) - 1);
        i1 = min(cam.w - 1, int(ceilf(umax + mu - 0.5f)) + 1);
        j0 = max(0, int(floorf(vmin - mv - 0.5f)) - 1);
        j1 = min(cam.h - 1, int(ceilf(vmax + mv - 0.5f)) + 1);
        return i0 <= i1 && j0 <= j1;
    }
    const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
    const float ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    return sphere_pixels(cx, cy, cz, 0.5f * sqrtf(ex * ex + ey * ey + ez * ez), cam, i0, i1, j0, j1);
}

// tiles (tx0, ty0, tx1, ty1) of a pixel rectangle
__device__ __forceinline__ int4 rect_tiles(int4 pr, int ts) {
    return pr.z < pr.x ? make_int4(0, 0, -1, -1) : make_int4(pr.x / ts, pr.y / ts, pr.z / ts, pr.w / ts);
}

// Per primitive: the pixel rectangle (i0, j0, i1, j1) of its volume of
// interest, empty (0, 0, -1, -1) when no pixel-centre ray can meet it, and
// the range of tiles (tx0, ty0, tx1, ty1) it is a candidate of.  Unless
// keep_all, that range is cut to the tiles of the rectangles of the subtree
// boxes on the other side of the primitive's first kKillLevels killing
// ancestors: in a tile that such a rectangle misses, the ancestor has no
// primitive of its other side (no pixel-centre ray of the tile meets those
// volumes of interest), so the primitive is dead there for the tile's hits
// and for every set that the pruning passes see.  (The cut is by whole
// tiles: the per-ray test still covers the primitive's whole rectangle in
// each tile it keeps.)
__global__ void __launch_bounds__(64) rect_count_kernel(const Voi* __restrict__ voi, DevCam cam, int ts,
                                                         const uint32_t* __restrict__ oside,
                                                         const float* __restrict__ sub, int keep_all, int tiles_x,
                                                         int4* __restrict__ rect, int4* __restrict__ trect,
                                                         uint32_t* __restrict__ tile_count) {
    // one wave per primitive p (a rectangle covers a few dozen tiles).  Eight
    // lanes: lane 0 the primitive's own rectangle, lane k (1..7) the k-th
    // killing ancestor's other side; the tile ranges are intersected across
    // the eight lanes and broadcast
    const int p = int(blockIdx.x), j = int(threadIdx.x & 7u);
    const bool lead = threadIdx.x < 8u;
    constexpr int kAll = 0x7FFFFFFF;
    int4 tr = make_int4(0, 0, kAll, kAll);
    if (lead && j == 0) {
        int i0, i1, j0, j1;
        const bool any = voi_pixels(voi[p], cam, i0, i1, j0, j1);
        const int4 pr = any ? make_int4(i0, j0, i1, j1) : make_int4(0, 0, -1, -1);
        if (threadIdx.x == 0) rect[p] = pr;
        tr = rect_tiles(pr, ts);
    } else if (lead && !keep_all) {
        const uint32_t other = oside[8 * size_t(p) + size_t(j - 1)];
        if (other != kNoKill) {
            int a0, a1, b0, b1;
            tr = aabb_pixels(sub + 8 * size_t(other), sub + 8 * size_t(other) + 3, cam, a0, a1, b0, b1)
                     ? rect_tiles(make_int4(a0, b0, a1, b1), ts) : make_int4(0, 0, -1, -1);
        }
    }
    for (int o = 1; o < 8; o <<= 1) {
        tr.x = max(tr.x, __shfl_xor(tr.x, o));
        tr.y = max(tr.y, __shfl_xor(tr.y, o));
        tr.z = min(tr.z, __shfl_xor(tr.z, o));
        tr.w = min(tr.w, __shfl_xor(tr.w, o));
    }
    tr.x = __builtin_amdgcn_readfirstlane(tr.x);
    tr.y = __builtin_amdgcn_readfirstlane(tr.y);
    tr.z = __builtin_amdgcn_readfirstlane(tr.z);
    tr.w = __builtin_amdgcn_readfirstlane(tr.w);
    if (!(tr.x <= tr.z && tr.y <= tr.w)) tr = make_int4(0, 0, -1, -1);
    if (threadIdx.x == 0) trect[p] = tr;
    // one candidate for every tile of the range
    const int w = tr.z - tr.x + 1, h = tr.w - tr.y + 1;
    if (w <= 0 || h <= 0) return;
    for (int k = int(threadIdx.x); k < w * h; k += int(blockDim.x))
        atomicAdd(tile_count + (tr.y + k / w) * tiles_x + tr.x + k % w, 1u);
}

// ---------------------------------------------------------------------------
// exclusive prefix sum of u32 (three passes, 1024-element blocks)
constexpr int kScanBlock = 1024;

__global__ void scan_block_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int n,
                                  uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t sh[kScanBlock];
    int base = blockIdx.x * kScanBlock;
    int i = base + threadIdx.x;
    uint32_t x = i < n ? in[i] : 0u;
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        uint32_t y = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += y;
        __syncthreads();
    }
    if (i < n) out[i] = sh[threadIdx.x] - x;
    if (threadIdx.x == kScanBlock - 1) block_sums[blockIdx.x] = sh[threadIdx.x];
}

__global__ void scan_sums_kernel(uint32_t* __restrict__ sums, int nb, uint32_t* __restrict__ total) {
    // single block, sequential chunks of 1024
    __shared__ uint32_t sh[kScanBlock];
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kScanBlock) {
        int i = base + threadIdx.x;
        uint32_t x = i < nb ? sums[i] : 0u;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < kScanBlock; off <<= 1) {
            uint32_t y = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
            __syncthreads();
            sh[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < nb) sums[i] = carry + sh[threadIdx.x] - x;
        uint32_t blk = sh[kScanBlock - 1];
        __syncthreads();
        carry += blk;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void scan_add_kernel(uint32_t* __restrict__ out, int n, const uint32_t* __restrict__ sums,
                                const uint32_t* __restrict__ total, uint32_t* __restrict__ out_total_slot) {
    int i = blockIdx.x * kScanBlock + threadIdx.x;
    if (i < n) out[i] += sums[blockIdx.x];
    if (i == 0 && out_total_slot) *out_total_slot = *total;
}

// One-workgroup exclusive scan for short arrays (the per-tile counts): chunks
// of 4 elements per thread, inclusive wave scans by shuffles, the sixteen
// wave totals scanned by one wave, a carry across chunks; two barriers per
// chunk of 4096 elements.
constexpr int kScanOneMax = 32768;

__global__ void __launch_bounds__(1024) scan_one_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                        int n, uint32_t* __restrict__ total,
                                                        uint32_t* __restrict__ out_total_slot) {
    __shared__ uint32_t wsum[16];
    const int tid = int(threadIdx.x), lane = tid & 63, w = tid >> 6;
    uint32_t carry = 0;
    for (int base = 0; base < n; base += 4096) {
        const int i0 = base + 4 * tid;
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; k++) v[k] = i0 + k < n ? in[i0 + k] : 0u;
        const uint32_t local = v[0] + v[1] + v[2] + v[3];
        uint32_t x = local;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = uint32_t(__shfl_up(int(x), o));
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        if (w == 0) {
            uint32_t t = lane < 16 ? wsum[lane] : 0u;
            for (int o = 1; o < 16; o <<= 1) {
                const uint32_t y = uint32_t(__shfl_up(int(t), o));
                if (lane >= o) t += y;
            }
            if (lane < 16) wsum[lane] = t;
        }
        __syncthreads();
        uint32_t run = carry + (w > 0 ? wsum[w - 1] : 0u) + x - local;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (i0 + k < n) out[i0 + k] = run;
            run += v[k];
        }
        carry += wsum[15];
        __syncthreads();   // wsum is rewritten by the next chunk
    }
    if (tid == 0) {
        *total = carry;
        if (out_total_slot) *out_total_slot = carry;
    }
}

// out[0..n) = exclusive scan of in, *total = sum; if out_total_slot, also
// writes the total there (CSR end offset).  scratch: >= ceil(n/1024)+1 u32.
void exclusive_scan(const uint32_t* in, uint32_t* out, int n, uint32_t* scratch, uint32_t* total,
                           uint32_t* out_total_slot, hipStream_t stream) {
    if (n <= kScanOneMax) {
        hipLaunchKernelGGL(scan_one_kernel, dim3(1), dim3(1024), 0, stream, in, out, n, total, out_total_slot);
        return;
    }
    int nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(scan_block_kernel, dim3(nb), dim3(kScanBlock), 0, stream, in, out, n, scratch);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanBlock), 0, stream, scratch, nb, total);
    hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(kScanBlock), 0, stream, out, n, scratch, total,
                       out_total_slot);
}

// ---------------------------------------------------------------------------
// candidate (primitive, tile) tests against the tiles' pixel-centre rays: one
// workgroup per primitive (its volume of interest is workgroup-uniform and
// read once), one wave per candidate tile in turn, each lane testing
// ts*ts/64 rays, then a wave min/max of the entry and exit depths
// number of lanes below this one whose bit is set in mask
__device__ __forceinline__ uint32_t lanes_below_mask(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

// Dispatch order of tiles: decreasing count of the candidates left for the
// per-ray test (the trace reuses the order).  The work of a tile grows with its
// count and a launch is set by its slowest workgroups, so the heavy tiles
// start first and the light ones fill the machine behind them.  One
// workgroup, counting sort over kOrderBuckets count buckets (counts beyond
// the last bucket share it); the order within a bucket is whatever the LDS
// atomics give, which changes only the schedule, not any result.  Most tiles
// of a sparse frame have no candidate left: the lanes of a wave that fall in
// that bucket take their places with one atomic per wave (ballot and rank),
// since thousands of lane atomics on one LDS word serialize.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 4 * kOrderThreads;
constexpr int kOrderBatch = 8;

__global__ void __launch_bounds__(kOrderThreads) tile_order_kernel(const uint32_t* __restrict__ tile_cnt,
                                                                    int n_tiles, uint32_t* __restrict__ order) {
    __shared__ uint32_t cnt[kOrderBuckets];
    __shared__ uint32_t part[kOrderThreads];
    constexpr uint32_t kEmpty = uint32_t(kOrderBuckets - 1);   // bucket of count 0
    const int tid = int(threadIdx.x);
    const bool leader = (tid & 63) == 0;
    auto bucket = [&](int t) {   // longest first
        const uint32_t len = t < n_tiles ? tile_cnt[t] : 0u;
        return kEmpty - min(len, kEmpty);
    };
    for (int b = tid; b < kOrderBuckets; b += kOrderThreads) cnt[b] = 0;
    __syncthreads();
    // the counts are read kOrderBatch per thread at a time, all loads issued
    // before the first atomic, so that one memory latency covers a batch
    for (int t0 = 0; t0 < n_tiles; t0 += kOrderThreads * kOrderBatch) {
        uint32_t bk[kOrderBatch];
#pragma unroll
        for (int k = 0; k < kOrderBatch; k++) bk[k] = bucket(t0 + k * kOrderThreads + tid);
#pragma unroll
        for (int k = 0; k < kOrderBatch; k++) {
            const bool in = t0 + k * kOrderThreads + tid < n_tiles;
            const uint64_t em = __ballot(in && bk[k] == kEmpty);
            if (in && bk[k] != kEmpty) atomicAdd(&cnt[bk[k]], 1u);
            if (leader && em) atomicAdd(&cnt[kEmpty], uint32_t(__popcll(em)));
        }
    }
    __syncthreads();
    // exclusive scan: four buckets per thread, then an inclusive scan of the
    // per-thread sums
    uint32_t c[4], sum = 0;
    for (int j = 0; j < 4; j++) { c[j] = cnt[4 * tid + j]; sum += c[j]; }
    part[tid] = sum;
    __syncthreads();
    for (int d = 1; d < kOrderThreads; d <<= 1) {
        uint32_t v = tid >= d ? part[tid - d] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = part[tid] - sum;
    for (int j = 0; j < 4; j++) { cnt[4 * tid + j] = run; run += c[j]; }
    __syncthreads();
    for (int t0 = 0; t0 < n_tiles; t0 += kOrderThreads * kOrderBatch) {
        uint32_t bk[kOrderBatch];
#pragma unroll
        for (int k = 0; k < kOrderBatch; k++) bk[k] = bucket(t0 + k * kOrderThreads + tid);
#pragma unroll
        for (int k = 0; k < kOrderBatch; k++) {
            const int t = t0 + k * kOrderThreads + tid;
            const bool in = t < n_tiles, empty = in && bk[k] == kEmpty;
            const uint64_t em = __ballot(empty);
            uint32_t base = 0;
            if (leader && em) base = atomicAdd(&cnt[kEmpty], uint32_t(__popcll(em)));
            base = __builtin_amdgcn_readlane(base, 0);
            if (empty) order[base + lanes_below_mask(em)] = uint32_t(t);
            else if (in) order[atomicAdd(&cnt[bk[k]], 1u)] = uint32_t(t);
        }
    }
}

// per primitive (one workgroup): its index into a slot of each tile segment
__global__ void __launch_bounds__(256) cand_scatter_kernel(const int4* __restrict__ trect, int tiles_x,
                                                           const uint32_t* __restrict__ tile_off,
                                                           uint32_t* __restrict__ cursor,
                                                           uint32_t* __restrict__ slot_prim) {
    const int4 rc = trect[blockIdx.x];
    const int w = rc.z - rc.x + 1, h = rc.w - rc.y + 1;
    if (w <= 0 || h <= 0) return;
    for (int k = int(threadIdx.x); k < w * h; k += int(blockDim.x)) {
        const int tile = (rc.y + k / w) * tiles_x + rc.x + k % w;
        slot_prim[tile_off[tile] + atomicAdd(cursor + tile, 1u)] = blockIdx.x;
    }
}

// wave reductions over the 64 lanes through DPP row shifts and broadcasts
// (no LDS round trips); the result is read from lane 63
__device__ __forceinline__ float dpp_min(float v) {
    const int inf = __float_as_int(__builtin_inff());
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(inf, __float_as_int(v), 0x111, 0xf, 0xf, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(inf, __float_as_int(v), 0x112, 0xf, 0xf, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(inf, __float_as_int(v), 0x114, 0xf, 0xf, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(inf, __float_as_int(v), 0x118, 0xf, 0xf, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(inf, __float_as_int(v), 0x142, 0xa, 0xf, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(inf, __float_as_int(v), 0x143, 0xc, 0xf, false)));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float dpp_max(float v) {
    const int ninf = __float_as_int(-__builtin_inff());
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(ninf, __float_as_int(v), 0x111, 0xf, 0xf, false)));
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(ninf, __float_as_int(v), 0x112, 0xf, 0xf, false)));
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(ninf, __float_as_int(v), 0x114, 0xf, 0xf, false)));
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(ninf, __float_as_int(v), 0x118, 0xf, 0xf, false)));
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(ninf, __float_as_int(v), 0x142, 0xa, 0xf, false)));
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(ninf, __float_as_int(v), 0x143, 0xc, 0xf, false)));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Per tile (one workgroup of 4 waves): the tile's TS x TS pixel-centre rays
// are built once, one 8x8 block of them per lane-slot (TS^2/64 per lane); the
// waves take the tile's candidates in turn and intersect every ray with the
// candidate's volume of interest, skipping the 8x8 blocks outside the pixel
// rectangle of its bounding sphere.  The slot gets the primitive's node and
// the padded [min entry, max exit] view depth over the rays that hit, or the
// empty interval (+inf, -inf).  Workgroups take the tiles in the given order
// (most candidates first: the longest segments start early instead of
// finishing the frame late).
// waves per tile: sixteen take a 16x16 or 32x32 tile's candidates in turn,
// so that the longest lists end early; an 8x8 tile (one ray per lane) has few
// candidates to share
// Waves per tile of the test, in workgroups of four waves: a tile's waves
// share nothing (no LDS, no barrier), and a workgroup of four finds room on a
// compute unit beside other kernels' workgroups (other frames' traces) where
// one of sixteen would wait for a quarter of a compute unit to drain.
constexpr uint32_t test_waves(int ts) { return ts == 8 ? 4u : 16u; }
constexpr uint32_t kTestWgWaves = 4;
constexpr uint32_t test_wgs(int ts) { return test_waves(ts) / kTestWgWaves; }   // workgroups per tile

template <int TS>
__global__ void __launch_bounds__(64 * kTestWgWaves) tile_test_kernel(const Voi* __restrict__ voi, const int4* __restrict__ rect,
                                                        const uint32_t* __restrict__ tile_off,
                                                        const uint32_t* __restrict__ tile_n,
                                                        const uint32_t* __restrict__ order, int tiles_x, DevCam cam,
                                                        uint32_t* __restrict__ e_node, float* __restrict__ e_zin,
                                                        float* __restrict__ e_zout) {
    constexpr int RPL = TS * TS / 64;   // rays per lane
    const int tile = int(order[blockIdx.x / test_wgs(TS)]);
    const uint32_t e0 = tile_off[tile], n = tile_n[tile];
    if (n == 0) return;
    const int lane = int(threadIdx.x & 63u);
    // the wave's index among the tile's test_waves(TS) waves
    const uint32_t w = (blockIdx.x % test_wgs(TS)) * kTestWgWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    float dir[RPL][3], cosv[RPL];
    bool ok[RPL];
    constexpr int BX = TS / 8;   // 8x8 blocks per tile row
#pragma unroll
    for (int r = 0; r < RPL; r++) {
        const int i = tx * TS + (r % BX) * 8 + (lane & 7), j = ty * TS + (r / BX) * 8 + (lane >> 3);
        ok[r] = i < cam.w && j < cam.h;
        const Ray ray = pixel_ray(cam, min(i, cam.w - 1), min(j, cam.h - 1));
        dir[r][0] = ray.d[0]; dir[r][1] = ray.d[1]; dir[r][2] = ray.d[2];
        cosv[r] = ray.cosv;
    }
    const float o[3] = {cam.eye[0], cam.eye[1], cam.eye[2]};
    for (uint32_t c = w; c < n; c += test_waves(TS)) {
        const uint32_t p = __builtin_amdgcn_readfirstlane(e_node[e0 + c]);
        const Voi v = voi[p];
        float zmin = __builtin_inff(), zmax = -__builtin_inff();
        const int4 pr = rect[p];   // the candidate's pixel rectangle
#pragma unroll
        for (int r = 0; r < RPL; r++) {
            const int bi = tx * TS + (r % BX) * 8, bj = ty * TS + (r / BX) * 8;
            if (bi + 7 < pr.x || bi > pr.z || bj + 7 < pr.y || bj > pr.w) continue;   // uniform
            float t0, t1;
            if (ok[r] && ray_voi(v, o, dir[r], t0, t1) && t1 >= 0.f) {
                t0 = fmaxf(t0, 0.f);
                zmin = fminf(zmin, t0 * cosv[r]);
                zmax = fmaxf(zmax, t1 * cosv[r]);
            }
        }
        zmin = dpp_min(zmin);
        zmax = dpp_max(zmax);
        if (lane == 0) {
            e_node[e0 + c] = __float_as_uint(v.v[21]);
            if (zmin <= zmax) {
                // conservative padding for FP32 rounding of the intervals
                const float pad = 2e-5f * fmaxf(fabsf(zmax), 1.0f);
                e_zin[e0 + c] = fmaxf(zmin - pad, 0.f);
                e_zout[e0 + c] = zmax + pad;
            } else {
                e_zin[e0 + c] = __builtin_inff();
                e_zout[e0 + c] = -__builtin_inff();
            }
        }
    }
}


// ---------------------------------------------------------------------------
// per-tile sort by (z_in, node) and largest depth overlap
__device__ __forceinline__ uint32_t f2key(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr int kSortThreads = 256;

// Bitonic sort of keys[0..np2) (u64) with a u32 payload, in place, by the
// whole workgroup.  Works on LDS or on global memory (the latter with the
// workgroup-scope fences that the barrier carries).
template <class K, class V>
__device__ void bitonic_wg(K* keys, V* vals, int np2) {
    for (int k = 2; k <= np2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < np2; i += blockDim.x) {
                int ixj = i ^ j;
                if (ixj > i) {
                    bool up = (i & k) == 0;
                    K a = keys[i], b = keys[ixj];
                    if ((a > b) == up) {
                        keys[i] = b; keys[ixj] = a;
                        if (vals) { V t = vals[i]; vals[i] = vals[ixj]; vals[ixj] = t; }
                    }
                }
            }
            __threadfence_block();
            __syncthreads();
        }
    }
}

template <class K>
__device__ int upper_bound_keys(const K* a, int n, K x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int m = (lo + hi) >> 1;
        if (a[m] <= x) lo = m + 1; else hi = m;
    }
    return lo;
}

// Sorts one tile's segment [e0, e1) given staging arrays (LDS or global),
// then computes the largest number of closed intervals sharing a point.
__device__ void sort_segment(uint64_t* keys, uint32_t* vals, uint32_t* zo_keys, uint32_t e0, uint32_t e1,
                             uint32_t* e_node, float* e_zin, float* e_zout, uint32_t* ovl_out) {
    int n = int(e1 - e0);
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (int i = threadIdx.x; i < np2; i += blockDim.x) {
        if (i < n) {
            keys[i] = (uint64_t(f2key(e_zin[e0 + i])) << 32) | e_node[e0 + i];
            vals[i] = __float_as_uint(e_zout[e0 + i]);
        } else {
            keys[i] = ~0ull;
            vals[i] = 0u;
        }
    }
    __threadfence_block();
    __syncthreads();
    bitonic_wg(keys, vals, np2);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        uint64_t k = keys[i];
        e_node[e0 + i] = uint32_t(k & 0xFFFFFFFFu);
        uint32_t zb = uint32_t(k >> 32);
        e_zin[e0 + i] = __uint_as_float((zb & 0x80000000u) ? (zb & 0x7FFFFFFFu) : ~zb);
        e_zout[e0 + i] = __uint_as_float(vals[i]);
    }
    __threadfence_block();
    __syncthreads();
    // exit depths sorted separately: overlap at z_in(i) = #(z_in <= z_in(i)) - #(z_out < z_in(i))
    for (int i = threadIdx.x; i < np2; i += blockDim.x) zo_keys[i] = i < n ? f2key(e_zout[e0 + i]) : 0xFFFFFFFFu;
    __threadfence_block();
    __syncthreads();
    bitonic_wg(zo_keys, (uint32_t*)nullptr, np2);
    uint32_t best = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        uint32_t zb = f2key(e_zin[e0 + i]);
        // #(z_in <= zb): keys sorted by z_in first
        uint64_t probe = (uint64_t(zb) << 32) | 0xFFFFFFFFull;
        int a = upper_bound_keys(keys, n, probe);
        // #(z_out < zb)
        int lo = 0, hi = n;
        while (lo < hi) {
            int m = (lo + hi) >> 1;
            if (zo_keys[m] < zb) lo = m + 1; else hi = m;
        }
        uint32_t ov = uint32_t(a - lo);
        best = best > ov ? best : ov;
    }
    // workgroup max
    __shared__ uint32_t red;
    if (threadIdx.x == 0) red = 0;
    __syncthreads();
    atomicMax(&red, best);
    __syncthreads();
    if (threadIdx.x == 0) *ovl_out = red;
}

// ---------------------------------------------------------------------------
// Tile-level pruning (not in the paper).  Every active set the tracer builds
// for a block of the tile is a subset of the tile's list, and a primitive that
// cannot reach the root for the whole list cannot for any subset of it: the
// set of primitives surviving the dead-primitive rule (a killing ancestor with
// no primitive of the set on its other side; repeated until nothing drops)
// only shrinks with the set, and removing a dead primitive leaves the pruned
// view unchanged.  So the entries of dead primitives are dropped once here and
// every subfrustum view stays what it was.  Per tile: the distinct primitives
// sorted by index, then rounds of (LCAs of consecutive primitives into a hash
// set, chain test, compaction), then a stable in-place compaction of the
// entries.  One workgroup per tile; lists up to kPruneLdsCap in LDS, longer
// ones in global scratch (7 words per entry).
constexpr int kPruneThreads = 256;
// words of a tile's statistics record: candidates tested, tested pixels by
// kind (3), tested candidates that hit, padding
constexpr int kTileStat = 8;
constexpr int kPruneLdsCap = 1024;
constexpr int kPruneBatch = kPruneLdsCap / kPruneThreads;   // keys per thread of rank_sort_wg

// exclusive rank of this thread among the workgroup's threads with keep set,
// in thread order; *total gets their count
__device__ int block_rank(bool keep, int* total) {
    __shared__ int wsum[kPruneThreads / 64];
    const int lane = int(threadIdx.x) & 63, w = int(threadIdx.x) >> 6;
    const uint64_t mk = __ballot(keep);
    if (lane == 0) wsum[w] = __popcll(mk);
    __syncthreads();
    int before = 0, all = 0;
    for (int k = 0; k < kPruneThreads / 64; k++) {
        before += k < w ? wsum[k] : 0;
        all += wsum[k];
    }
    __syncthreads();
    *total = all;
    return before + int(lanes_below_mask(mk));
}

// Sorts the keys of in[0..n) (in 16-byte aligned) other than 0xFFFFFFFF (distinct node indices)
// into out[0..count) by rank counting: each thread ranks its kPruneBatch
// keys against all n in one pass, and every lane reads the same in[j] at the
// same time (an LDS broadcast).  n <= kPruneThreads * kPruneBatch.  A list of
// a few hundred takes one pass of n steps where a bitonic network of
// workgroup barriers took 45 or more barrier stages.
__device__ void rank_sort_wg(const uint32_t* in, int n, uint32_t* out) {
    const int tid = int(threadIdx.x);
    uint32_t x[kPruneBatch], r[kPruneBatch];
#pragma unroll
    for (int k = 0; k < kPruneBatch; k++) {
        const int i = tid + k * kPruneThreads;
        x[k] = i < n ? in[i] : 0xFFFFFFFFu;
        r[k] = 0;
    }
    // four keys per LDS read (in is 16-byte aligned), four reads in flight
    int j = 0;
#pragma unroll 4
    for (; j + 4 <= n; j += 4) {
        const uint4 y = *reinterpret_cast<const uint4*>(in + j);
#pragma unroll
        for (int k = 0; k < kPruneBatch; k++)
            r[k] += (y.x < x[k] ? 1u : 0u) + (y.y < x[k] ? 1u : 0u) + (y.z < x[k] ? 1u : 0u) + (y.w < x[k] ? 1u : 0u);
    }
    for (; j < n; j++) {
        const uint32_t y = in[j];
#pragma unroll
        for (int k = 0; k < kPruneBatch; k++) r[k] += y < x[k] ? 1u : 0u;
    }
#pragma unroll
    for (int k = 0; k < kPruneBatch; k++)
        if (x[k] != 0xFFFFFFFFu) out[r[k]] = x[k];
    __threadfence_block();
    __syncthreads();
}

// Removes from the sorted node list cur[0..m) the primitives that are dead for
// the set (a killing ancestor with no primitive of the set on its other
// side), repeating until nothing drops; nxt (m words) and tab (2^bits words,
// 2^bits >= 2m) are scratch.  cur ends pointing at the survivors (sorted);
// returns their count.
__device__ int dead_rounds(uint32_t*& cur, uint32_t* nxt, int m, uint32_t* tab, int bits,
                           const uint32_t* __restrict__ rmq, const uint4* __restrict__ kslot,
                           const uint32_t* __restrict__ kill, uint32_t n_nodes) {
    const int tid = int(threadIdx.x);
    for (int round = 0; round < 32 && m > 0; round++) {
        for (int i = tid; i < (1 << bits); i += kPruneThreads) tab[i] = kNoKill;
        __threadfence_block();
        __syncthreads();
        for (int i = tid; i < m - 1; i += kPruneThreads) {
            const uint32_t x = cur[i], y = cur[i + 1];
            const uint32_t l = (x < y && y < n_nodes) ? lca_query(rmq, n_nodes, x, y) : 0u;
            hinsert(tab, bits, l);
        }
        __threadfence_block();
        __syncthreads();
        int kept = 0;
        for (int c = 0; c < m; c += kPruneThreads) {
            const int i = c + tid;
            const uint32_t x = i < m ? cur[i] : 0u;
            const bool keep = i < m && chain_alive(x, kslot, kill, n_nodes, tab, bits);
            int tot;
            const int r = block_rank(keep, &tot);
            if (keep) nxt[kept + r] = x;
            kept += tot;
        }
        __threadfence_block();
        __syncthreads();
        const bool changed = kept < m;
        uint32_t* t = cur;
        cur = nxt;
        nxt = t;
        m = kept;
        if (!changed) break;
    }
    return m;
}

// Compacts the candidate segment [e0, e0 + n) in place to the entries that
// hit (non-empty interval) and, unless keep_all, whose primitive survives the
// rule for the set of hits; a (2^ceil(log2 n) words), b (n words) and tab
// (2^bits words, 2^bits >= 2n) are scratch.  Returns the number kept; *hits
// gets the number of hits.
__device__ int prune_tile(uint32_t e0, int n, uint32_t* e_node, float* e_zin, float* e_zout, uint32_t* a,
                          uint32_t* b, uint32_t* tab, int bits, const uint32_t* __restrict__ rmq,
                          const uint4* __restrict__ kslot, const uint32_t* __restrict__ kill, uint32_t n_nodes,
                          bool keep_all, int* hits) {
    const int tid = int(threadIdx.x);
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    // the primitives that hit, sorted (misses and padding sort last)
    int m = 0;   // primitives are distinct within a tile's segment
    for (int c = 0; c < np2; c += kPruneThreads) {
        const int i = c + tid;
        const bool hit = i < n && e_zin[e0 + i] <= e_zout[e0 + i];
        if (i < np2) a[i] = hit ? e_node[e0 + i] : 0xFFFFFFFFu;
        int tot;
        block_rank(hit, &tot);
        m += tot;
    }
    *hits = m;
    __threadfence_block();
    __syncthreads();
    uint32_t* cur = a;
    if (!keep_all) {
        uint32_t* nxt = b;
        if (n <= kPruneThreads * kPruneBatch) {   // the sorted hits go to b (m <= n words)
            rank_sort_wg(a, n, b);
            cur = b;
            nxt = a;
        } else {
            bitonic_wg(a, (uint32_t*)nullptr, np2);
        }
        m = dead_rounds(cur, nxt, m, tab, bits, rmq, kslot, kill, n_nodes);
    }
    // the survivors, as a hash set; then the entries, compacted in place in
    // their order (each chunk is read whole before any of it is written)
    if (!keep_all) {
        for (int i = tid; i < (1 << bits); i += kPruneThreads) tab[i] = kNoKill;
        __threadfence_block();
        __syncthreads();
        for (int i = tid; i < m; i += kPruneThreads) hinsert(tab, bits, cur[i]);
        __threadfence_block();
        __syncthreads();
    }
    int kept = 0;
    for (int c = 0; c < n; c += kPruneThreads) {
        const int i = c + tid;
        const bool in = i < n;
        const uint32_t x = in ? e_node[e0 + i] : 0u;
        const float zi = in ? e_zin[e0 + i] : 0.f, zo = in ? e_zout[e0 + i] : 0.f;
        const bool keep = in && zi <= zo && (keep_all || (m > 0 && hfind(tab, bits, x, tab[hslot(x, bits)])));
        int tot;
        const int r = block_rank(keep, &tot);   // its barriers separate the reads from the writes
        if (keep) {
            e_node[e0 + kept + r] = x;
            e_zin[e0 + kept + r] = zi;
            e_zout[e0 + kept + r] = zo;
        }
        kept += tot;
        __threadfence_block();
        __syncthreads();
    }
    return kept;
}

__device__ __forceinline__ int prune_bits(int n) {   // 2^bits >= 2n, and > 2(n - 1)
    int bits = 1;
    while ((1 << bits) < 2 * n) bits++;
    return bits;
}

// Drops, before the per-ray test, the candidates of a tile that are dead for
// the tile's whole candidate set.  A primitive dead for a set is dead for any
// subset of it (its killing ancestor has no partner there either), and the
// set of primitives alive for the hits is alive for every set between them
// and the hits, so the entries kept after the test are unchanged.  Segments
// longer than the LDS capacity, and keep_all builds, keep every candidate.
// The segment is compacted in place (order kept) and tile_n gets its length.
// The tile's record gets the candidates kept ([0]) and, by kind, the pixels
// of their rectangles inside the tile ([1..3], the work of the per-ray test).
__device__ void add_tested(const uint32_t* slot_prim, uint32_t e0, int n, int tile, int tiles_x, int ts,
                           const int4* __restrict__ rect, const Voi* __restrict__ voi, uint32_t* __restrict__ tstat) {
    __shared__ unsigned long long part[kPruneThreads / 64][3];
    const int tid = int(threadIdx.x), lane = tid & 63, w = tid >> 6;
    const int x0 = (tile % tiles_x) * ts, y0 = (tile / tiles_x) * ts;
    unsigned long long area[3] = {0, 0, 0};
    for (int i = tid; i < n; i += kPruneThreads) {
        const uint32_t p = slot_prim[e0 + i];
        const int4 r = rect[p];
        const int wx = min(r.z, x0 + ts - 1) - max(r.x, x0) + 1, wy = min(r.w, y0 + ts - 1) - max(r.y, y0) + 1;
        const int kind = int(voi[p].v[20]) - ST_SPHERE;
        if (wx > 0 && wy > 0 && kind >= 0 && kind < 3) area[kind] += (unsigned long long)(wx * wy);
    }
    for (int k = 0; k < 3; k++) {
        for (int o = 32; o > 0; o >>= 1) area[k] += __shfl_xor(area[k], o);
        if (lane == 0) part[w][k] = area[k];
    }
    __syncthreads();
    // the tile's record (summed only for a build that reports statistics)
    if (tid < 3) {
        unsigned long long t = 0;
        for (int k = 0; k < kPruneThreads / 64; k++) t += part[k][tid];
        tstat[kTileStat * size_t(tile) + 1 + tid] = uint32_t(t);
    }
    if (tid == 0) tstat[kTileStat * size_t(tile)] = uint32_t(n);
}

// ---------------------------------------------------------------------------
// One wave per tile for lists of at most 64 entries (nearly every tile): the
// same rule as prune_tile / dead_rounds, with the set in registers (lane i
// holds one primitive), the order by rank counting and the compaction by
// ballot, and a 128-slot LDS hash set per wave; no workgroup barrier.
constexpr int kWavePruneMax = 64;
constexpr int kWavePruneBits = 7;   // 128 slots >= 2 x 64

__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Whether the lane's primitive x (valid when in) survives the dead-primitive
// rule for the set of the valid lanes' primitives (distinct nodes), applied
// until nothing drops.  srt (64 words) and tab (128 words) are the wave's LDS
// scratch.  Must be called by every lane of the wave, in uniform control flow
// (never behind a lane-dependent condition such as a short-circuit &&): it
// clears the table lane by lane and reads neighbouring lanes' registers.
__device__ bool wave_alive(uint32_t x, bool in, uint32_t* srt, uint32_t* tab, const uint32_t* __restrict__ rmq,
                           const uint4* __restrict__ kslot, const uint32_t* __restrict__ kill, uint32_t n_nodes) {
    const int lane = int(threadIdx.x & 63u);
    const uint64_t vm = __ballot(in);
    int m = __popcll(vm);
    if (m == 0) return false;
    // sorted set: rank of each valid node among the valid nodes
    uint32_t rank = 0;
    for (uint64_t left = vm; left; left &= left - 1) {
        const uint32_t xj = __builtin_amdgcn_readlane(x, int(__builtin_ctzll(left)));
        rank += xj < x ? 1u : 0u;
    }
    if (in) srt[rank] = x;
    wsync();
    uint32_t sx = lane < m ? srt[lane] : 0xFFFFFFFFu;
    for (int round = 0; round < 32; round++) {
        // the nodes with set members on both sides: LCAs of consecutive members
        tab[lane] = kNoKill;
        tab[lane + 64] = kNoKill;
        wsync();
        const uint32_t nx = __shfl_down(sx, 1);
        // (the order check only guards the table reads against a logic error)
        if (lane < m - 1 && sx < nx && nx < n_nodes) hinsert(tab, kWavePruneBits, lca_query(rmq, n_nodes, sx, nx));
        wsync();
        const bool keep = lane < m && chain_alive(sx, kslot, kill, n_nodes, tab, kWavePruneBits);
        const uint64_t km = __ballot(keep);
        const int k = __popcll(km);
        if (k == m) break;
        wsync();
        if (keep) srt[lanes_below_mask(km)] = sx;
        wsync();
        m = k;
        sx = lane < m ? srt[lane] : 0xFFFFFFFFu;
        if (m == 0) break;
    }
    // membership of x in the surviving set
    wsync();
    tab[lane] = kNoKill;
    tab[lane + 64] = kNoKill;
    wsync();
    if (lane < m) hinsert(tab, kWavePruneBits, sx);
    wsync();
    return in && m > 0 && hfind(tab, kWavePruneBits, x, tab[hslot(x, kWavePruneBits)]);
}

// Pre-test pruning of a tile with 1..64 candidates by one wave: same result
// as the workgroup path (cand_prune_wg).  srt (64 words) and tab (128 words)
// are the wave's LDS scratch.
__device__ void cand_prune_wave(int tile, uint32_t e0, int n, int tiles_x, int ts, const uint32_t* __restrict__ prims,
                                const int4* __restrict__ rect, const Voi* __restrict__ voi, uint32_t* slot_prim,
                                uint32_t* __restrict__ tile_n, const uint32_t* __restrict__ rmq,
                                const uint4* __restrict__ kslot, const uint32_t* __restrict__ kill, uint32_t n_nodes,
                                uint32_t* __restrict__ tstat, uint32_t* srt, uint32_t* tab) {
    const int lane = int(threadIdx.x & 63u);
    const bool in = lane < n;
    const uint32_t p = in ? slot_prim[e0 + lane] : 0u;
    const uint32_t x = in ? prims[p] : 0u;
    const bool keep = wave_alive(x, in, srt, tab, rmq, kslot, kill, n_nodes);
    const uint64_t km = __ballot(keep);
    if (keep) slot_prim[e0 + lanes_below_mask(km)] = p;   // every lane read its slot above
    const int kept = __popcll(km);
    // the tile's record: candidates kept, and by kind the pixels of their
    // rectangles inside the tile (the per-ray test's work)
    const int x0 = (tile % tiles_x) * ts, y0 = (tile / tiles_x) * ts;
    uint32_t area[3] = {0, 0, 0};
    if (keep) {
        const int4 r = rect[p];
        const int wx = min(r.z, x0 + ts - 1) - max(r.x, x0) + 1, wy = min(r.w, y0 + ts - 1) - max(r.y, y0) + 1;
        const int kind = int(voi[p].v[20]) - ST_SPHERE;
        if (wx > 0 && wy > 0 && kind >= 0 && kind < 3) area[kind] = uint32_t(wx * wy);
    }
    for (int k = 0; k < 3; k++)
        for (int o = 32; o > 0; o >>= 1) area[k] += uint32_t(__shfl_xor(int(area[k]), o));
    if (lane == 0) {
        tile_n[tile] = uint32_t(kept);
        tstat[kTileStat * size_t(tile)] = uint32_t(kept);
        for (int k = 0; k < 3; k++) tstat[kTileStat * size_t(tile) + 1 + k] = area[k];
    }
}

// Post-test pruning of a tile with 1..64 tested candidates by one wave: same
// result as prune_tile (entries that hit and survive, compacted in order).
// srt (64 words) and tab (128 words) are the wave's LDS scratch.
__device__ void tile_prune_wave(int tile, uint32_t e0, int n, uint32_t* e_node, float* e_zin, float* e_zout,
                                uint32_t* __restrict__ tile_cnt, const uint32_t* __restrict__ rmq,
                                const uint4* __restrict__ kslot, const uint32_t* __restrict__ kill, uint32_t n_nodes,
                                int keep_all, uint32_t* __restrict__ tstat, uint32_t* srt, uint32_t* tab) {
    const int lane = int(threadIdx.x & 63u);
    const bool in = lane < n;
    const uint32_t x = in ? e_node[e0 + lane] : 0u;
    const float zi = in ? e_zin[e0 + lane] : 0.f, zo = in ? e_zout[e0 + lane] : 0.f;
    const bool hit = in && zi <= zo;
    bool keep = hit;
    if (!keep_all) {   // uniform: every lane of the wave takes part in wave_alive
        const bool alive = wave_alive(x, hit, srt, tab, rmq, kslot, kill, n_nodes);
        keep = hit && alive;
    }
    const uint64_t km = __ballot(keep);
    const uint64_t hm = __ballot(hit);
    if (keep) {   // every lane read its entry above
        const uint32_t d = e0 + lanes_below_mask(km);
        e_node[d] = x;
        e_zin[d] = zi;
        e_zout[d] = zo;
    }
    if (lane == 0) {
        tile_cnt[tile] = uint32_t(__popcll(km));
        tstat[kTileStat * size_t(tile) + 4] = uint32_t(__popcll(hm));
    }
}

// Work split of the two pruning kernels (one workgroup per tile in the
// grid): wave w of workgroup b takes tile 4b + w when its list is empty or
// short (nearly every tile; one wave, no barrier), and workgroup b takes tile
// b when its list is longer (the whole workgroup).  Four short tiles per
// workgroup keep four waves busy where a workgroup per short tile would hold
// its LDS for one, and the long lists, which sit next to each other around
// the clusters of a scene, still run side by side in their own workgroups.
constexpr int kPruneTiles = kPruneThreads / 64;

// Pre-test pruning of a tile with more than kWavePruneMax candidates (or
// keep_all) by the whole workgroup; a, b, tab are its LDS scratch.
__device__ void cand_prune_wg(int tile, uint32_t e0, int n, int tiles_x, int ts, const uint32_t* __restrict__ prims,
                              const int4* __restrict__ rect, const Voi* __restrict__ voi, uint32_t* slot_prim,
                              uint32_t* __restrict__ tile_n, const uint32_t* __restrict__ rmq,
                              const uint4* __restrict__ kslot, const uint32_t* __restrict__ kill, uint32_t n_nodes,
                              int keep_all, uint32_t* __restrict__ tstat, uint32_t* a, uint32_t* b, uint32_t* tab) {
    const int tid = int(threadIdx.x);
    if (n > kPruneLdsCap || keep_all) {
        if (tid == 0) tile_n[tile] = uint32_t(n);
        add_tested(slot_prim, e0, n, tile, tiles_x, ts, rect, voi, tstat);
        return;
    }
    {   // the thread's candidates: every slot load issued, then every node load
        uint32_t p[kPruneBatch];
#pragma unroll
        for (int k = 0; k < kPruneBatch; k++) {
            const int i = tid + k * kPruneThreads;
            p[k] = i < n ? slot_prim[e0 + i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kPruneBatch; k++) {
            const int i = tid + k * kPruneThreads;
            if (i < n) a[i] = prims[p[k]];
        }
    }
    __threadfence_block();
    __syncthreads();
    rank_sort_wg(a, n, b);   // n <= kPruneLdsCap
    const int bits = prune_bits(n);
    uint32_t* cur = b;
    const int m = dead_rounds(cur, a, n, tab, bits, rmq, kslot, kill, n_nodes);
    for (int i = tid; i < (1 << bits); i += kPruneThreads) tab[i] = kNoKill;
    __threadfence_block();
    __syncthreads();
    for (int i = tid; i < m; i += kPruneThreads) hinsert(tab, bits, cur[i]);
    __threadfence_block();
    __syncthreads();
    int kept = 0;
    for (int c = 0; c < n; c += kPruneThreads) {
        const int i = c + tid;
        const uint32_t p = i < n ? slot_prim[e0 + i] : 0u;
        const uint32_t x = i < n ? prims[p] : 0u;
        const bool keep = i < n && m > 0 && hfind(tab, bits, x, tab[hslot(x, bits)]);
        int tot;
        const int r = block_rank(keep, &tot);   // its barriers separate the reads from the writes
        if (keep) slot_prim[e0 + kept + r] = p;
        kept += tot;
        __threadfence_block();
        __syncthreads();
    }
    if (tid == 0) tile_n[tile] = uint32_t(kept);
    if (kept) add_tested(slot_prim, e0, kept, tile, tiles_x, ts, rect, voi, tstat);
}

__global__ void __launch_bounds__(kPruneThreads) cand_prune_kernel(
        const uint32_t* __restrict__ tile_off, int n_tiles, int tiles_x, int ts, const uint32_t* __restrict__ prims,
        const int4* __restrict__ rect, const Voi* __restrict__ voi, uint32_t* slot_prim, uint32_t* __restrict__ tile_n,
        const uint32_t* __restrict__ rmq, const uint4* __restrict__ kslot, const uint32_t* __restrict__ kill,
        uint32_t n_nodes, int keep_all, uint32_t* __restrict__ tstat) {
    __shared__ __align__(16) uint32_t a[kPruneLdsCap], b[kPruneLdsCap], tab[2 * kPruneLdsCap];
    const int w = int(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));   // wave-uniform
    // the wave's tile, if empty or short (its scratch: 64 words of a, 128 of tab)
    const int mine = int(blockIdx.x) * kPruneTiles + w;
    if (mine < n_tiles) {
        const uint32_t e0 = tile_off[mine];
        const int n = int(tile_off[mine + 1] - e0);
        if (n == 0) {
            if ((threadIdx.x & 63u) == 0) tile_n[mine] = 0u;
        } else if (!keep_all && n <= kWavePruneMax) {
            cand_prune_wave(mine, e0, n, tiles_x, ts, prims, rect, voi, slot_prim, tile_n, rmq, kslot, kill, n_nodes,
                            tstat, a + 64 * w, tab + 128 * w);
        }
    }
    // the workgroup's tile, if its list is longer (uniform: every thread reads
    // the same offsets, which this kernel does not write)
    const int tile = int(blockIdx.x);
    if (tile >= n_tiles) return;
    const uint32_t e0 = tile_off[tile];
    const int n = int(tile_off[tile + 1] - e0);
    if (n == 0 || (!keep_all && n <= kWavePruneMax)) return;
    __syncthreads();   // the waves are done with their scratch
    cand_prune_wg(tile, e0, n, tiles_x, ts, prims, rect, voi, slot_prim, tile_n, rmq, kslot, kill, n_nodes, keep_all,
                  tstat, a, b, tab);
}

// tstat[kTileStat * t] holds tile t's candidate count after the pre-test
// pruning (the count the per-ray test takes): this kernel decides from it,
// since it rewrites tile_cnt while other workgroups still decide
__global__ void __launch_bounds__(kPruneThreads) tile_prune_kernel(
        const uint32_t* __restrict__ tile_off, int n_tiles, uint32_t* e_node, float* e_zin, float* e_zout,
        uint32_t* __restrict__ tile_cnt, uint32_t* __restrict__ long_list, uint32_t* __restrict__ misc,
        const uint32_t* __restrict__ rmq, const uint4* __restrict__ kslot, const uint32_t* __restrict__ kill,
        uint32_t n_nodes, int keep_all, uint32_t* __restrict__ tstat) {
    __shared__ __align__(16) uint32_t a[kPruneLdsCap], b[kPruneLdsCap], tab[2 * kPruneLdsCap];
    const int w = int(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));   // wave-uniform
    // the wave's tile, if its list is short (its scratch: 64 words of a, 128 of tab)
    const int mine = int(blockIdx.x) * kPruneTiles + w;
    if (mine < n_tiles) {
        const int n = int(tstat[kTileStat * size_t(mine)]);
        if (n > 0 && n <= kWavePruneMax)
            tile_prune_wave(mine, tile_off[mine], n, e_node, e_zin, e_zout, tile_cnt, rmq, kslot, kill, n_nodes,
                            keep_all, tstat, a + 64 * w, tab + 128 * w);
    }
    // the workgroup's tile, if its list is longer (uniform)
    const int tile = int(blockIdx.x);
    if (tile >= n_tiles) return;
    const int n = int(tstat[kTileStat * size_t(tile)]);
    if (n <= kWavePruneMax) return;
    if (n > kPruneLdsCap) {   // for the long-list kernel
        if (threadIdx.x == 0) long_list[atomicAdd(misc + 5, 1u)] = uint32_t(tile);
        return;
    }
    __syncthreads();   // the waves are done with their scratch
    int hits;
    const int kept = prune_tile(tile_off[tile], n, e_node, e_zin, e_zout, a, b, tab, prune_bits(n), rmq, kslot, kill,
                                n_nodes, keep_all != 0, &hits);
    if (threadIdx.x == 0) {
        tile_cnt[tile] = uint32_t(kept);
        tstat[kTileStat * size_t(tile) + 4] = uint32_t(hits);
    }
}

// long lists: scratch in global memory, 7 words per entry of the segment
// (a: 2n >= 2^ceil(log2 n), b: n, tab: 4n >= 2^bits)
__global__ void __launch_bounds__(kPruneThreads) tile_prune_long_kernel(
        const uint32_t* __restrict__ tile_off, uint32_t* e_node, float* e_zin, float* e_zout,
        uint32_t* __restrict__ tile_cnt, const uint32_t* __restrict__ long_list, const uint32_t* __restrict__ misc,
        uint32_t* scratch, const uint32_t* __restrict__ rmq, const uint4* __restrict__ kslot,
        const uint32_t* __restrict__ kill, uint32_t n_nodes, int keep_all, uint32_t* __restrict__ tstat) {
    const uint32_t n_long = misc[5];
    for (uint32_t idx = blockIdx.x; idx < n_long; idx += gridDim.x) {
        const uint32_t tile = long_list[idx];
        const uint32_t e0 = tile_off[tile];
        const int n = int(tile_cnt[tile]);   // tested candidates of the segment
        __syncthreads();
        uint32_t* base = scratch + size_t(7) * e0;
        int hits;
        const int kept = prune_tile(e0, n, e_node, e_zin, e_zout, base, base + 2 * n, base + 3 * n, prune_bits(n),
                                    rmq, kslot, kill, n_nodes, keep_all != 0, &hits);
        if (threadIdx.x == 0) {
            tile_cnt[tile] = uint32_t(kept);
            tstat[kTileStat * size_t(tile) + 4] = uint32_t(hits);
        }
        __syncthreads();
    }
}

constexpr int kSortLdsCap = 1024;

// Short lists (up to 64 entries), one wave per tile, four tiles per
// workgroup, no barriers: each lane holds one entry; its position in
// (z_in, node) order is the number of smaller keys, and its depth overlap the
// number of entries entering at or before its entry depth minus those that
// exit before it (the same counts the workgroup sort takes from its sorted
// arrays).  Longer lists are queued for tile_sort_kernel.
__global__ void __launch_bounds__(256) tile_sort_short_kernel(
        const uint32_t* __restrict__ tile_off, const uint32_t* __restrict__ tile_cnt, int n_tiles, uint32_t* e_node,
        float* e_zin, float* e_zout, uint32_t* __restrict__ tile_ovl, uint32_t* __restrict__ queue,
        uint32_t* __restrict__ misc, uint32_t ma_fast, uint32_t* __restrict__ wide) {
    const int lane = int(threadIdx.x & 63u);
    const int tile = int(blockIdx.x) * 4 + int(threadIdx.x >> 6);
    if (tile >= n_tiles) return;   // whole waves
    const uint32_t e0 = tile_off[tile], n = tile_cnt[tile];
    if (n == 0) {
        if (lane == 0) tile_ovl[tile] = 0;
        return;
    }
    if (n > 64u) {
        if (lane == 0) queue[atomicAdd(misc + 10, 1u)] = uint32_t(tile);
        return;
    }
    const bool in = uint32_t(lane) < n;
    const uint32_t node = in ? e_node[e0 + lane] : 0u;
    const float zi = in ? e_zin[e0 + lane] : 0.f, zo = in ? e_zout[e0 + lane] : 0.f;
    const uint32_t ki = f2key(zi), ko = f2key(zo);
    uint32_t rank = 0, a = 0, lo = 0;
    for (int j = 0; j < int(n); j++) {
        const uint32_t kj = __builtin_amdgcn_readlane(ki, j), nj = __builtin_amdgcn_readlane(node, j);
        const uint32_t oj = __builtin_amdgcn_readlane(ko, j);
        rank += (kj < ki || (kj == ki && nj < node)) ? 1u : 0u;
        a += kj <= ki ? 1u : 0u;
        lo += oj < ki ? 1u : 0u;
    }
    if (in) {   // every lane has read its entry above
        e_node[e0 + rank] = node;
        e_zin[e0 + rank] = zi;
        e_zout[e0 + rank] = zo;
    }
    uint32_t ov = in ? a - lo : 0u;
    for (int o = 32; o > 0; o >>= 1) ov = max(ov, uint32_t(__shfl_xor(int(ov), o)));
    if (lane == 0) {
        tile_ovl[tile] = ov;
        if (ov > ma_fast) wide[1 + atomicAdd(wide, 1u)] = uint32_t(tile);
    }
}

// Queued lists (more than 64 entries), a workgroup per tile in turn; lists
// longer than kSortLdsCap go on to the long list.
__global__ void __launch_bounds__(kSortThreads) tile_sort_kernel(
        const uint32_t* __restrict__ tile_off, const uint32_t* __restrict__ tile_cnt, uint32_t* e_node,
        float* e_zin, float* e_zout, uint32_t* __restrict__ tile_ovl, const uint32_t* __restrict__ queue,
        uint32_t* __restrict__ long_list, uint32_t* __restrict__ misc, uint32_t ma_fast, uint32_t* __restrict__ wide) {
    __shared__ uint64_t keys[kSortLdsCap];
    __shared__ uint32_t vals[kSortLdsCap];
    __shared__ uint32_t zo[kSortLdsCap];
    __shared__ uint32_t ov;
    const uint32_t n_queued = misc[10];
    for (uint32_t idx = blockIdx.x; idx < n_queued; idx += gridDim.x) {
        const uint32_t tile = queue[idx];
        const uint32_t e0 = tile_off[tile], e1 = e0 + tile_cnt[tile];
        const uint32_t n = e1 - e0;
        if (n > uint32_t(kSortLdsCap)) {
            if (threadIdx.x == 0) long_list[atomicAdd(misc + 0, 1u)] = tile;
        } else {
            sort_segment(keys, vals, zo, e0, e1, e_node, e_zin, e_zout, &ov);
            if (threadIdx.x == 0) {
                tile_ovl[tile] = ov;
                if (ov > ma_fast) wide[1 + atomicAdd(wide, 1u)] = tile;
            }
        }
        __syncthreads();
    }
}

// long lists: bitonic sort in global scratch (one workgroup per long tile)
__global__ void __launch_bounds__(kSortThreads) tile_sort_long_kernel(
        const uint32_t* __restrict__ tile_off, const uint32_t* __restrict__ tile_cnt, uint32_t* e_node, float* e_zin,
        float* e_zout,
        uint32_t* __restrict__ tile_ovl, const uint32_t* __restrict__ long_list, uint32_t* __restrict__ misc,
        uint64_t* scratch_keys, uint32_t* scratch_vals, uint32_t* scratch_zo, uint32_t ma_fast,
        uint32_t* __restrict__ wide) {
    uint32_t n_long = misc[0];
    __shared__ uint32_t ov;
    for (uint32_t idx = blockIdx.x; idx < n_long; idx += gridDim.x) {
        uint32_t tile = long_list[idx];
        uint32_t e0 = tile_off[tile], e1 = e0 + tile_cnt[tile];
        // scratch segment: entries of this tile padded to a power of two fit
        // in [2*e0, 2*e0 + 2n) since np2 < 2n
        uint64_t* k = scratch_keys + 2 * size_t(e0);
        uint32_t* v = scratch_vals + 2 * size_t(e0);
        uint32_t* z = scratch_zo + 2 * size_t(e0);
        sort_segment(k, v, z, e0, e1, e_node, e_zin, e_zout, &ov);
        if (threadIdx.x == 0) {
            tile_ovl[tile] = ov;
            if (ov > ma_fast) wide[1 + atomicAdd(wide, 1u)] = tile;
        }
        __syncthreads();
    }
}


// ---------------------------------------------------------------------------
st_status launch_voi(st_scene* s, hipStream_t stream) {
    int P = s->n_prims;
    hipLaunchKernelGGL(voi_kernel, dim3((P + 255) / 256), dim3(256), 0, stream, s->d_prims, P, s->d_par,
                       s->d_roi, s->d_blob, s->d_voi);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ST_OK : device_error(e, "voi_kernel");
}

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// clears device words with a kernel (graph-capture safe, unlike memset nodes)
__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t n, uint32_t v) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Statistics of a build that reports them, from the per-tile records and
// arrays (one workgroup, no contended atomics during the build): misc[1] the
// largest depth overlap, misc[2] the longest kept list, misc[3] the kept
// entries, misc[6] the tested candidates that hit, misc[7] the candidates
// tested, pix[kind] the pixels tested.
constexpr int kStatThreads = 1024;
__global__ void __launch_bounds__(kStatThreads) build_stats_kernel(const uint32_t* __restrict__ tile_cnt,
                                                                   const uint32_t* __restrict__ tile_ovl,
                                                                   const uint32_t* __restrict__ tstat, int n_tiles,
                                                                   uint32_t* __restrict__ misc,
                                                                   unsigned long long* __restrict__ pix) {
    __shared__ unsigned long long part[kStatThreads / 64][7];
    const int tid = int(threadIdx.x), lane = tid & 63, w = tid >> 6;
    // largest overlap, longest list, kept entries, tested candidates, tested pixels by kind
    unsigned long long v[7] = {0, 0, 0, 0, 0, 0, 0};
    unsigned long long hits = 0;
    for (int t = tid; t < n_tiles; t += kStatThreads) {
        const uint32_t* r = tstat + kTileStat * size_t(t);
        v[0] = max(v[0], (unsigned long long)tile_ovl[t]);
        v[1] = max(v[1], (unsigned long long)tile_cnt[t]);
        v[2] += tile_cnt[t];
        v[3] += r[0];
        v[4] += r[1];
        v[5] += r[2];
        v[6] += r[3];
        hits += r[4];
    }
    for (int k = 0; k < 7; k++)
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long x = __shfl_xor(v[k], o);
            v[k] = k < 2 ? max(v[k], x) : v[k] + x;
        }
    for (int o = 32; o > 0; o >>= 1) hits += __shfl_xor(hits, o);
    __shared__ unsigned long long phits[kStatThreads / 64];
    if (lane == 0) {
        for (int k = 0; k < 7; k++) part[w][k] = v[k];
        phits[w] = hits;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long r[7] = {0, 0, 0, 0, 0, 0, 0}, h = 0;
        for (int q = 0; q < kStatThreads / 64; q++) {
            for (int k = 0; k < 7; k++) r[k] = k < 2 ? max(r[k], part[q][k]) : r[k] + part[q][k];
            h += phits[q];
        }
        misc[1] = uint32_t(r[0]);
        misc[2] = uint32_t(r[1]);
        misc[3] = uint32_t(r[2]);
        misc[6] = uint32_t(h);
        misc[7] = uint32_t(r[3]);
        pix[0] = r[4];
        pix[1] = r[5];
        pix[2] = r[6];
    }
}

// clears the counters of a build in one launch: tile counts (T + 1 words),
// scatter cursors (T), misc (64), the wide-list length (1) and the tiles'
// statistics records (kTileStat T)
__global__ void clear_build_kernel(uint32_t* __restrict__ tcnt, uint32_t* __restrict__ cur, uint32_t T,
                                   uint32_t* __restrict__ misc, uint32_t* __restrict__ wide,
                                   uint32_t* __restrict__ tstat) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < uint32_t(kTileStat) * T) tstat[i] = 0u;
    if (i <= T) tcnt[i] = 0u;
    if (i < T) cur[i] = 0u;
    if (i < 64u) misc[i] = 0u;
    if (i == 0u) wide[0] = 0u;
}

hipError_t fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

// replay: the same kernel sequence for an unchanged scene, camera and tuning,
// reusing the sizes and buffers of the previous build (the counts are
// deterministic): no host synchronization, no allocation, no memset nodes.
st_status build_abuffer_device(st_scene* s, const st_tuning& t, hipStream_t stream, bool replay) {
    const int P = s->n_prims;
    const int T = s->n_tiles;
    const int ts = t.tile;
    // scratch layout (bytes): pixel rectangles P*16, tile ranges P*16, scan
    // sums, tile counts (T+1)*4, cursors T*4, long list T*4, sort queue T*4,
    // tile statistics records T*4*kTileStat, misc 64*4
    size_t nb_t = size_t(T + kScanBlock) / kScanBlock + 2;
    size_t off_rect = 0;
    size_t off_trect = align_up(off_rect + size_t(P) * 16);
    size_t off_sums = align_up(off_trect + size_t(P) * 16);
    size_t off_tcnt = align_up(off_sums + nb_t * 4 + 16);
    size_t off_cur = align_up(off_tcnt + size_t(T + 1) * 4);
    size_t off_long = align_up(off_cur + size_t(T) * 4);
    size_t off_queue = align_up(off_long + size_t(T) * 4);
    size_t off_tstat = align_up(off_queue + size_t(T) * 4);
    size_t off_misc = align_up(off_tstat + size_t(T) * 4 * kTileStat);
    size_t need = align_up(off_misc + 64 * 4);
    if (replay && (need > s->scratch_bytes || !s->ab_valid)) {
        set_error("build replay: no previous build of this size");
        return ST_E_STALE;
    }
    if (need > s->scratch_bytes) {
        if (s->d_scratch) dev_free(s, s->d_scratch, stream);
        s->d_scratch = dev_alloc(s, need, stream);
        if (!s->d_scratch) { s->scratch_bytes = 0; set_error("build: scratch allocation failed"); return ST_E_NOMEM; }
        s->scratch_bytes = need;
    }
    char* base = (char*)s->d_scratch;
    int4* rect = (int4*)(base + off_rect);
    int4* trect = (int4*)(base + off_trect);
    uint32_t* sums = (uint32_t*)(base + off_sums);
    uint32_t* tcnt = (uint32_t*)(base + off_tcnt);
    uint32_t* cur = (uint32_t*)(base + off_cur);
    uint32_t* longl = (uint32_t*)(base + off_long);
    uint32_t* tstat = (uint32_t*)(base + off_tstat);   // per tile: kTileStat words
    uint32_t* queue = (uint32_t*)(base + off_queue);   // lists of more than 64 entries (count misc[10])
    uint32_t* misc = (uint32_t*)(base + off_misc);
    hipError_t e;
#define ST_CHECK(x, what) do { e = (x); if (e != hipSuccess) return device_error(e, what); } while (0)

    hipLaunchKernelGGL(clear_build_kernel, dim3((uint32_t(kTileStat) * uint32_t(T) + 64u) / 256u + 1u), dim3(256), 0,
                       stream, tcnt, cur, uint32_t(T), misc, s->d_wide, tstat);
    unsigned long long* pix = reinterpret_cast<unsigned long long*>(misc + 16);   // 3 counters, 8-byte aligned
    // pixel rectangle, tile range and candidate count of every primitive
    if (P) hipLaunchKernelGGL(rect_count_kernel, dim3(P), dim3(64), 0, stream, s->d_voi, s->dcam, ts, s->d_oside,
                              s->d_sub, t.keep_all_entries, s->tiles_x, rect, trect, tcnt);
    exclusive_scan(tcnt, s->d_tile_off, T, sums, misc + 9, s->d_tile_off + T, stream);
    uint32_t n_cand = replay ? s->n_cand : 0u;
    if (!replay) {
        ST_CHECK(hipMemcpyAsync(&n_cand, misc + 9, 4, hipMemcpyDeviceToHost, stream), "copy candidate count");
        ST_CHECK(hipStreamSynchronize(stream), "sync (candidates)");
        s->n_cand = n_cand;
    }

    // candidate slots = entry arrays (grown on demand)
    if (int64_t(n_cand) > s->ab_cap) {
        dev_free(s, s->d_e_node, stream);
        dev_free(s, s->d_e_zin, stream);
        dev_free(s, s->d_e_zout, stream);
        int64_t cap = std::max<int64_t>(int64_t(n_cand) + int64_t(n_cand) / 4, 1024);
        s->d_e_node = (uint32_t*)dev_alloc(s, size_t(cap) * 4, stream);
        s->d_e_zin = (float*)dev_alloc(s, size_t(cap) * 4, stream);
        s->d_e_zout = (float*)dev_alloc(s, size_t(cap) * 4, stream);
        if (!s->d_e_node || !s->d_e_zin || !s->d_e_zout) {
            set_error("build: A-buffer allocation failed");
            s->ab_cap = 0;
            return ST_E_NOMEM;
        }
        s->ab_cap = cap;
    }
    if (P && n_cand)
        hipLaunchKernelGGL(cand_scatter_kernel, dim3(P), dim3(256), 0, stream, trect, s->tiles_x, s->d_tile_off,
                           cur, s->d_e_node);
    // candidates dead for their tile's candidate set: dropped before the test
    // (d_tile_cnt: candidates left per tile)
    hipLaunchKernelGGL(cand_prune_kernel, dim3(T), dim3(kPruneThreads), 0, stream, s->d_tile_off, T, s->tiles_x, ts,
                       s->d_prims, rect, s->d_voi, s->d_e_node, s->d_tile_cnt, s->d_rmq,
                       reinterpret_cast<const uint4*>(s->d_kslot), s->d_kill, uint32_t(s->n_nodes),
                       t.keep_all_entries, tstat);
    // order by candidates left, for the test and for the trace.  Every build
    // writes it, also one without candidates (all counts zero: the identity
    // up to bucket order), because the trace reads it for every block.
    hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(kOrderThreads), 0, stream, s->d_tile_cnt, T,
                       s->d_tile_order);
    if (P && n_cand) {
        hipEvent_t* ev = nullptr;
        if (s->time_test) {   // a fresh pair per launch (created once, reused after a restart)
            if (s->test_used * 2 + 2 > s->test_events.size()) {
                hipEvent_t a = nullptr, b = nullptr;
                ST_CHECK(hipEventCreate(&a), "timing event");
                ST_CHECK(hipEventCreate(&b), "timing event");
                s->test_events.push_back(a);
                s->test_events.push_back(b);
            }
            ev = &s->test_events[s->test_used * 2];
            s->test_used++;
            ST_CHECK(hipEventRecord(ev[0], stream), "timing record");
        }
        if (ts == 8)
            hipLaunchKernelGGL(tile_test_kernel<8>, dim3(T * test_wgs(8)), dim3(64 * kTestWgWaves), 0, stream, s->d_voi, rect, s->d_tile_off,
                               s->d_tile_cnt, s->d_tile_order, s->tiles_x, s->dcam, s->d_e_node, s->d_e_zin, s->d_e_zout);
        else if (ts == 16)
            hipLaunchKernelGGL(tile_test_kernel<16>, dim3(T * test_wgs(16)), dim3(64 * kTestWgWaves), 0, stream, s->d_voi, rect, s->d_tile_off,
                               s->d_tile_cnt, s->d_tile_order, s->tiles_x, s->dcam, s->d_e_node, s->d_e_zin, s->d_e_zout);
        else
            hipLaunchKernelGGL(tile_test_kernel<32>, dim3(T * test_wgs(32)), dim3(64 * kTestWgWaves), 0, stream, s->d_voi, rect, s->d_tile_off,
                               s->d_tile_cnt, s->d_tile_order, s->tiles_x, s->dcam, s->d_e_node, s->d_e_zin, s->d_e_zout);
        if (ev) ST_CHECK(hipEventRecord(ev[1], stream), "timing record");
    }
    const uint32_t n_ent = n_cand;   // slots the pruning and the sorts work on
    // scratch of the long lists (pruning: 7 words per entry; sorting: 2
    // padded copies of key, value and exit depth, 16 bytes per entry each)
    size_t long_bytes = size_t(2) * n_ent * (8 + 4 + 4) + 64;
    if (long_bytes > s->long_bytes) {
        dev_free(s, s->d_long, stream);
        s->d_long = dev_alloc(s, long_bytes + long_bytes / 4, stream);
        s->long_bytes = s->d_long ? long_bytes + long_bytes / 4 : 0;
        if (!s->d_long) { set_error("build: sort scratch allocation failed"); return ST_E_NOMEM; }
    }
    char* lbuf = (char*)s->d_long;
    // tile-level pruning (long lists: the kernel reads their count on the device)
    hipLaunchKernelGGL(tile_prune_kernel, dim3(T), dim3(kPruneThreads), 0, stream, s->d_tile_off, T, s->d_e_node,
                       s->d_e_zin, s->d_e_zout, s->d_tile_cnt, longl, misc, s->d_rmq,
                       reinterpret_cast<const uint4*>(s->d_kslot), s->d_kill, uint32_t(s->n_nodes),
                       t.keep_all_entries, tstat);
    // A replay has the counts of its sizing build: kernels whose queue was
    // empty then are not launched (three launches of a few microseconds each
    // on frames without long lists).
    if (!replay || s->n_long_prune)
        hipLaunchKernelGGL(tile_prune_long_kernel, dim3(std::min(T, 512)), dim3(kPruneThreads), 0, stream,
                       s->d_tile_off, s->d_e_node, s->d_e_zin, s->d_e_zout, s->d_tile_cnt, longl, misc,
                       reinterpret_cast<uint32_t*>(lbuf), s->d_rmq, reinterpret_cast<const uint4*>(s->d_kslot),
                       s->d_kill, uint32_t(s->n_nodes), t.keep_all_entries, tstat);
    hipLaunchKernelGGL(tile_sort_short_kernel, dim3((T + 3) / 4), dim3(256), 0, stream, s->d_tile_off,
                       s->d_tile_cnt, T, s->d_e_node, s->d_e_zin, s->d_e_zout, s->d_tile_ovl, queue, misc,
                       uint32_t(s->ab_ma_fast), s->d_wide);
    if (!replay || s->n_sort_queue)
        hipLaunchKernelGGL(tile_sort_kernel, dim3(std::min(T, 512)), dim3(kSortThreads), 0, stream, s->d_tile_off,
                       s->d_tile_cnt, s->d_e_node, s->d_e_zin, s->d_e_zout, s->d_tile_ovl, queue, longl, misc,
                       uint32_t(s->ab_ma_fast), s->d_wide);
    // long tiles, if any (the kernel reads their count on the device)
    uint64_t* sk = (uint64_t*)lbuf;
    uint32_t* sv = (uint32_t*)(lbuf + size_t(2) * n_ent * 8);
    uint32_t* sz = (uint32_t*)(lbuf + size_t(2) * n_ent * 12);
    if (!replay || s->n_long_sort)
        hipLaunchKernelGGL(tile_sort_long_kernel, dim3(std::min(T, 512)), dim3(kSortThreads), 0, stream,
                       s->d_tile_off, s->d_tile_cnt, s->d_e_node, s->d_e_zin, s->d_e_zout, s->d_tile_ovl, longl,
                       misc, sk, sv, sz, uint32_t(s->ab_ma_fast), s->d_wide);
    // (the trace takes the tiles in the test's order: a tile's kept entries
    // grow with its tested candidates, and a second ordering pass costs more
    // than it gains)
    if (replay) {
        e = hipGetLastError();
        return e == hipSuccess ? ST_OK : device_error(e, "binning kernels");
    }
    hipLaunchKernelGGL(build_stats_kernel, dim3(1), dim3(kStatThreads), 0, stream, s->d_tile_cnt, s->d_tile_ovl, tstat,
                       T, misc, pix);
    uint32_t h_misc[16] = {}, h_wide = 0;
    ST_CHECK(hipMemcpyAsync(h_misc, misc, 64, hipMemcpyDeviceToHost, stream), "copy build stats");
    ST_CHECK(hipMemcpyAsync(s->cand_pix, pix, 24, hipMemcpyDeviceToHost, stream), "copy candidate pixels");
    ST_CHECK(hipMemcpyAsync(&h_wide, s->d_wide, 4, hipMemcpyDeviceToHost, stream), "copy wide count");
    e = hipGetLastError();
    if (e != hipSuccess) return device_error(e, "binning kernels");
    ST_CHECK(hipStreamSynchronize(stream), "sync (build)");
    s->max_overlap = h_misc[1];
    s->max_list = h_misc[2];
    s->n_live = h_misc[3];
    s->n_entries = h_misc[6];   // candidates that hit
    s->n_tested = h_misc[7];    // candidates left for the per-ray test
    s->n_long_sort = h_misc[0];   // queue lengths of the long-list kernels
    s->n_long_prune = h_misc[5];
    s->n_sort_queue = h_misc[10];
    s->n_wide = h_wide;
#undef ST_CHECK
    return ST_OK;
}

}  // namespace st
