// Ablation variants of the paper's Table 1 (ParentPtr/Full and FastPtr/Full):
// the rendering without synchronization, for comparison with the
// synchronized path.  A full-resolution dexel buffer holds, for every pixel,
// the primitives whose volume of interest its ray meets with the ray's own
// entry and exit t (the paper's A-buffer at pixel resolution), sorted by
// primitive address.  Every ray is then traced on its own: it walks the
// events of its list, and in each interval with a fixed set of active
// primitives it sphere-traces with the field evaluated directly by the sparse
// bottom-up traversal of Algorithm 1 (parent or fast ancestor pointers,
// st_sparse.h) at every step.  No pruned view is built and nothing is shared
// between the rays of a wave.  The stepping rules (probe, bracket refinement,
// forward-mode normal) are the synchronized tracer's.
#include <algorithm>
#include <cstring>
#include <string>

#include "st_field.h"
#include "st_internal.h"
#include "st_sparse.h"
#include "st_voi.h"
#include "st_trace.h"

namespace st {

namespace {

struct DexelArgs {
    DevCam cam;
    int ts, tiles_x;
    const uint32_t* tile_off;
    const uint32_t* tile_cnt;
    const uint32_t* e_node;
    const uint32_t* pslot;
    const Voi* voi;
    const uint32_t* pix_off;   // fill pass: CSR offsets per pixel
    uint32_t* pix_cnt;         // count pass output
    uint32_t* d_node;          // fill pass outputs, per pixel sorted by node
    float* d_tin;
    float* d_tout;
};

// One thread per pixel, one wave per 8x8 block (the block lies in one tile,
// so the tile's list is read with uniform addresses).  count: the number of
// list entries whose volume of interest the pixel's ray meets; fill: those
// entries with the ray's own [t_in, t_out] (clamped at the eye, padded for
// FP32 rounding as at binning), inserted in increasing node order.
template <bool Fill>
__global__ void __launch_bounds__(64) dexel_kernel(DexelArgs A) {
    const int lane = int(threadIdx.x);
    const int px = int(blockIdx.x) * 8 + (lane & 7), py = int(blockIdx.y) * 8 + (lane >> 3);
    if (px >= A.cam.w || py >= A.cam.h) return;
    const size_t pix = size_t(py) * size_t(A.cam.w) + size_t(px);
    const int tile = (py / A.ts) * A.tiles_x + px / A.ts;
    const uint32_t e0 = A.tile_off[tile], n = A.tile_cnt[tile];
    const Ray ray = pixel_ray(A.cam, px, py);
    const float o[3] = {A.cam.eye[0], A.cam.eye[1], A.cam.eye[2]};
    uint32_t cnt = 0;
    const uint32_t base = Fill ? A.pix_off[pix] : 0u;
    for (uint32_t c = 0; c < n; c++) {
        const uint32_t node = A.e_node[e0 + c];
        const Voi v = A.voi[A.pslot[node]];
        float t0, t1;
        if (!(ray_voi(v, o, ray.d, t0, t1) && t1 >= 0.f)) continue;
        if constexpr (Fill) {
            const float pad = 2e-5f * fmaxf(fabsf(t1), 1.0f);
            const float a = fmaxf(fmaxf(t0, 0.f) - pad, 0.f), b = t1 + pad;
            uint32_t j = cnt;
            while (j > 0 && A.d_node[base + j - 1] > node) {
                A.d_node[base + j] = A.d_node[base + j - 1];
                A.d_tin[base + j] = A.d_tin[base + j - 1];
                A.d_tout[base + j] = A.d_tout[base + j - 1];
                j--;
            }
            A.d_node[base + j] = node;
            A.d_tin[base + j] = a;
            A.d_tout[base + j] = b;
        }
        cnt++;
    }
    if constexpr (!Fill) A.pix_cnt[pix] = cnt;
}

struct AblArgs {
    DevCam cam;
    const uint32_t* blob;
    const uint32_t* anc;       // fast ancestor pointers (fast variant)
    const NodePar* par;
    const uint32_t* pix_off;
    const uint32_t* d_node;
    const float* d_tin;
    const float* d_tout;
    float eps, probe, probe_cap, lip_fixed;
    int max_steps, refine_iters;
    float* out_depth;
    float* out_normal;
    unsigned long long* wrec;   // per 8x8 block: kWaveStats counters
};

struct AblTree {
    const uint32_t* bl;
    const uint32_t* fast;
    bool use_fast;
    __device__ uint32_t blob(uint32_t n) const { return bl[n]; }
    __device__ uint32_t anc(uint32_t n) const { return use_fast ? fast[n] : blob_anc(bl[n]); }
};

// Active primitives of the ray's current interval: the entries of its list
// (in node order) whose [t_in, t_out) holds the interval's start.
struct AblAct {
    const uint32_t* node;
    const float* tin;
    const float* tout;
    uint32_t i, end;
    float t;
    __device__ bool next(uint32_t& n) {
        while (i < end) {
            const uint32_t k = i++;
            if (tin[k] <= t && tout[k] > t) {
                n = node[k];
                return true;
            }
        }
        return false;
    }
};

struct ValL {
    float v, L;
};

// field value and Lipschitz bound of the evaluated expression; +inf marks an
// unused branch (no operator then contributes its factor)
struct EvalF {
    typedef ValL V;
    const uint32_t* blob;
    const NodePar* par;
    P3<float> p;
    uint32_t* kinds;   // node evaluations by class (sphere, box, capsule, operator)
    uint32_t sm = 0;
    __device__ V none() const { return {__builtin_inff(), 0.f}; }
    __device__ V prim(uint32_t n) {
        const uint32_t k = blob_op(blob[n]);
        count_class(*reinterpret_cast<uint32_t(*)[4]>(kinds), k);
        return {prim_eval<float>(k, (const cfloat*)(par[n].v), p), 1.f};
    }
    __device__ V single(uint32_t op, const V& a, bool from_left) const {
        return single_passes(blob[op], from_left) ? a : none();
    }
    __device__ V op(uint32_t op, const V& a, const V& b) {
        if (a.v == __builtin_inff()) return single(op, b, false);
        if (b.v == __builtin_inff()) return single(op, a, true);
        kinds[3]++;
        const cfloat* q = (const cfloat*)(par[op].v);
        return {op_eval<float>(blob_op(blob[op]), q, a.v, b.v, sm), q[4] * fmaxf(a.L, b.L)};
    }
};

struct EvalG {
    typedef Dual V;
    const uint32_t* blob;
    const NodePar* par;
    P3<Dual> p;
    uint32_t sm = 0;
    __device__ V none() const { return {__builtin_inff(), 0.f, 0.f, 0.f}; }
    __device__ V prim(uint32_t n) const {
        return prim_eval<Dual>(blob_op(blob[n]), (const cfloat*)(par[n].v), p);
    }
    __device__ V single(uint32_t op, const V& a, bool from_left) const {
        return single_passes(blob[op], from_left) ? a : none();
    }
    __device__ V op(uint32_t op, const V& a, const V& b) {
        if (a.v == __builtin_inff()) return single(op, b, false);
        if (b.v == __builtin_inff()) return single(op, a, true);
        return op_eval<Dual>(blob_op(blob[op]), (const cfloat*)(par[op].v), a, b, sm);
    }
};

template <bool Fast>
__global__ void __launch_bounds__(64) ablation_trace_kernel(AblArgs A) {
    const int lane = int(threadIdx.x);
    const int px = int(blockIdx.x) * 8 + (lane & 7), py = int(blockIdx.y) * 8 + (lane >> 3);
    const bool valid = px < A.cam.w && py < A.cam.h;
    const AblTree tr{A.blob, A.anc, Fast};
    uint32_t kinds[4] = {0, 0, 0, 0};
    uint32_t evals = 0, gevals = 0, steps = 0, visited = 0, n_seg = 0;
    bool hit = false, unconv = false, overflow = false;
    float t_hit = __builtin_inff(), nx = 0.f, ny = 0.f, nz = 0.f;
    if (valid) {
        const size_t pix = size_t(py) * size_t(A.cam.w) + size_t(px);
        const uint32_t o0 = A.pix_off[pix], o1 = A.pix_off[pix + 1];
        const Ray ray = pixel_ray(A.cam, px, py);
        float t = 0.f;
        float tp = 0.f, vp = 0.f, hp = 0.f;
        bool tp_ok = false, last_safe = true;
        // every interval starts at an event of the list (an entry or exit)
        // that lies after the previous start: at most 2 (o1 - o0) intervals
        for (uint32_t guard = 2u * (o1 - o0) + 2u; guard > 0u && !hit && !unconv && !overflow; guard--) {
            // active set at t and the next event after t
            bool any = false;
            float te = __builtin_inff(), tn_in = __builtin_inff();
            for (uint32_t k = o0; k < o1; k++) {
                const float a = A.d_tin[k], b = A.d_tout[k];
                if (a <= t && b > t) { any = true; te = fminf(te, b); }
                else if (a > t) { te = fminf(te, a); tn_in = fminf(tn_in, a); }
            }
            if (!any) {
                if (!(tn_in < __builtin_inff())) break;   // no volume of interest ahead: miss
                t = tn_in;
                tp_ok = false;
                continue;
            }
            n_seg++;
            const float ta = t;
            AblAct act0{A.d_node, A.d_tin, A.d_tout, o0, o1, ta};
            int mode = 1;   // 1 trace, 2 refine
            float ra = 0.f, fa = 0.f, rb = 0.f, fb = 0.f;
            int nref = 0, side = 0;
            while (mode != 0) {
                const P3<float> p{fmaf(t, ray.d[0], ray.o[0]), fmaf(t, ray.d[1], ray.o[1]), fmaf(t, ray.d[2], ray.o[2])};
                AblAct act = act0;
                EvalF ev{A.blob, A.par, p, kinds};
                const ValL r = sparse_traverse<Fast, kStack>(tr, act, ev, visited, overflow);
                evals++;
                if (overflow) break;
                const float v = r.v;
                if (mode == 1) {
                    steps++;
                    if (v <= 0.f) {
                        if (!tp_ok || last_safe) {
                            t_hit = t;
                            hit = true;
                            mode = 0;
                        } else {
                            ra = tp; fa = vp; rb = t; fb = v;
                            nref = 0; side = 0;
                            mode = 2;
                            t = ra + (rb - ra) * (fa / (fa - fb));
                            if (!(t > ra && t < rb)) t = 0.5f * (ra + rb);
                        }
                        continue;
                    }
                    // +inf: no surface in this interval (root unused)
                    const float L = A.lip_fixed > 0.f ? A.lip_fixed : r.L;
                    const float safe_s = v == __builtin_inff() ? te - t : v / L;
                    float s = safe_s;
                    if (!(safe_s >= A.probe)) {
                        s = probe_len(v, t, tp, vp, tp_ok, hp, A.eps, A.probe_cap, safe_s);
                        hp = fminf(s, te - t);   // the step taken (clamped at te below)
                    } else {
                        hp = 0.f;
                    }
                    last_safe = !(s > safe_s);
                    tp = t; vp = v; tp_ok = v < __builtin_inff();
                    const float tn = t + s;
                    if (tn >= te) {
                        t = te;
                        mode = 0;
                    } else if (int(steps) >= A.max_steps) {
                        unconv = true;
                        mode = 0;
                    } else {
                        t = tn;
                    }
                } else {
                    nref++;
                    if (v <= 0.f) {
                        rb = t; fb = v;
                        if (side == -1) fa *= 0.5f;
                        side = -1;
                    } else {
                        ra = t; fa = v;
                        if (side == 1) fb *= 0.5f;
                        side = 1;
                    }
                    if (nref >= A.refine_iters || rb - ra <= 1e-6f * fmaxf(1.f, rb)) {
                        t_hit = ra + (rb - ra) * (fa / (fa - fb));
                        if (!(t_hit >= ra && t_hit <= rb)) t_hit = rb;
                        hit = true;
                        mode = 0;
                    } else {
                        t = ra + (rb - ra) * (fa / (fa - fb));
                        if (!(t > ra && t < rb)) t = 0.5f * (ra + rb);
                    }
                }
            }
            if (hit) {
                const P3<Dual> p = make_point(fmaf(t_hit, ray.d[0], ray.o[0]), fmaf(t_hit, ray.d[1], ray.o[1]),
                                              fmaf(t_hit, ray.d[2], ray.o[2]), Dual{});
                AblAct act = act0;
                EvalG ev{A.blob, A.par, p};
                const Dual g = sparse_traverse<Fast, kStack>(tr, act, ev, visited, overflow);
                const float gn = sqrtf(g.gx * g.gx + g.gy * g.gy + g.gz * g.gz);
                const float ig = gn > 0.f ? 1.0f / gn : 0.f;
                nx = g.gx * ig; ny = g.gy * ig; nz = g.gz * ig;
                gevals++;
            }
        }
        A.out_depth[pix] = hit ? t_hit : __builtin_inff();
        A.out_normal[3 * pix + 0] = hit ? nx : 0.f;
        A.out_normal[3 * pix + 1] = hit ? ny : 0.f;
        A.out_normal[3 * pix + 2] = hit ? nz : 0.f;
    }
    // counters of the block (same record layout as the synchronized trace)
    unsigned long long v[kWaveStats] = {};
    v[S_RAYS] = __popcll(ballot(valid));
    v[S_HITS] = __popcll(ballot(valid && hit));
    v[S_UNCONV] = __popcll(ballot(valid && unconv));
    v[S_EVALS] = wave_sum(evals + gevals);
    v[S_GEVALS] = wave_sum(gevals);
    v[S_STEPS] = wave_sum(steps);
    for (int q = 0; q < 4; q++) v[S_NODE + q] = wave_sum(kinds[q]);
    v[S_SUBF] = wave_sum(n_seg);
    v[S_VIEWN] = wave_sum(visited);   // operators the traversals visited
    v[S_STALL] = __popcll(ballot(valid && overflow));
    unsigned long long mine = 0;
#pragma unroll
    for (int c = 0; c < kWaveStats; c++) mine = lane == c ? v[c] : mine;
    const size_t rec = size_t(blockIdx.y) * gridDim.x + blockIdx.x;
    if (lane < kWaveStats) A.wrec[rec * kWaveStats + size_t(lane)] = mine;
}

}  // namespace

// dexel buffer of the current A-buffer (count, scan, one host
// synchronization for the size, fill)
static st_status build_dexels(st_scene* s, hipStream_t stream) {
    const int W = s->dcam.w, H = s->dcam.h;
    const size_t npix = size_t(W) * size_t(H);
    const size_t nb = (npix + 1023) / 1024 + 2;
    const size_t need_off = (npix + 1) * 4 + npix * 4 + nb * 4 + 64;
    if (need_off > s->dx_meta_bytes) {
        dev_free(s, s->d_dx_meta, stream);
        s->d_dx_meta = dev_alloc(s, need_off, stream);
        s->dx_meta_bytes = s->d_dx_meta ? need_off : 0;
        if (!s->d_dx_meta) { set_error("ablation: dexel offsets allocation failed"); return ST_E_NOMEM; }
    }
    uint32_t* off = static_cast<uint32_t*>(s->d_dx_meta);
    uint32_t* cnt = off + npix + 1;
    uint32_t* sums = cnt + npix;
    uint32_t* total = sums + nb;
    DexelArgs D{};
    D.cam = s->dcam;
    D.ts = s->ab_tune.tile;
    D.tiles_x = s->tiles_x;
    D.tile_off = s->d_tile_off;
    D.tile_cnt = s->d_tile_cnt;
    D.e_node = s->d_e_node;
    D.pslot = s->d_pslot;
    D.voi = s->d_voi;
    D.pix_cnt = cnt;
    const dim3 grid((W + 7) / 8, (H + 7) / 8);
    hipLaunchKernelGGL(dexel_kernel<false>, grid, dim3(64), 0, stream, D);
    exclusive_scan(cnt, off, int(npix), sums, total, off + npix, stream);
    uint32_t n_dx = 0;
    hipError_t e = hipMemcpyAsync(&n_dx, total, 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_error(e, "ablation: dexel count");
    const size_t need = size_t(std::max<uint32_t>(n_dx, 1u)) * 12 + 512;
    if (need > s->dx_bytes) {
        dev_free(s, s->d_dx, stream);
        s->d_dx = dev_alloc(s, need, stream);
        s->dx_bytes = s->d_dx ? need : 0;
        if (!s->d_dx) { set_error("ablation: dexel buffer allocation failed"); return ST_E_NOMEM; }
    }
    s->n_dexels = n_dx;
    const size_t cap = (need - 512) / 12;
    D.pix_off = off;
    D.d_node = static_cast<uint32_t*>(s->d_dx);
    D.d_tin = reinterpret_cast<float*>(D.d_node + cap);
    D.d_tout = D.d_tin + cap;
    hipLaunchKernelGGL(dexel_kernel<true>, grid, dim3(64), 0, stream, D);
    e = hipGetLastError();
    return e == hipSuccess ? ST_OK : device_error(e, "ablation: dexel kernels");
}

}  // namespace st

using namespace st;

extern "C" st_status st_trace_ablation(st_scene* s, const st_camera* cam, int32_t variant, float* out_depth,
                                       float* out_normal, st_stats* out_stats, void* stream_v) {
    if (!s || !cam || !out_depth || !out_normal) { set_error("ablation: NULL argument"); return ST_E_INVALID; }
    if (variant != ST_ABLATION_PARENT_PTR && variant != ST_ABLATION_FAST_PTR) {
        set_error("ablation: variant must be ST_ABLATION_PARENT_PTR or ST_ABLATION_FAST_PTR");
        return ST_E_INVALID;
    }
    hipStream_t stream = (hipStream_t)stream_v;
    if (!s->ab_valid || std::memcmp(cam, &s->ab_cam, sizeof(st_camera)) != 0) {
        set_error("ablation: the A-buffer was not built for this camera");
        return ST_E_STALE;
    }
    st_status r = build_dexels(s, stream);
    if (r != ST_OK) return r;
    const int W = s->dcam.w, H = s->dcam.h;
    const dim3 grid((W + 7) / 8, (H + 7) / 8);
    const uint32_t n_blocks = grid.x * grid.y;
    const size_t rec_bytes = size_t(n_blocks) * kWaveStats * 8u;
    if (rec_bytes > s->wrec_bytes) {
        dev_free(s, s->d_wrec, stream);
        s->d_wrec = dev_alloc(s, rec_bytes, stream);
        s->wrec_bytes = s->d_wrec ? rec_bytes : 0;
        if (!s->d_wrec) { set_error("ablation: counter record allocation failed"); return ST_E_NOMEM; }
    }
    const st_tuning& t = s->ab_tune;
    const size_t cap = (s->dx_bytes - 512) / 12;
    AblArgs A{};
    A.cam = s->dcam;
    A.blob = s->d_blob;
    A.anc = s->d_fast;
    A.par = s->d_par;
    A.pix_off = static_cast<const uint32_t*>(s->d_dx_meta);
    A.d_node = static_cast<const uint32_t*>(s->d_dx);
    A.d_tin = reinterpret_cast<const float*>(A.d_node + cap);
    A.d_tout = A.d_tin + cap;
    A.eps = t.eps;
    A.probe = std::max(t.probe_step, t.eps);
    A.probe_cap = kProbeCapFactor * A.probe;
    A.lip_fixed = t.lipschitz;
    A.max_steps = t.max_steps;
    A.refine_iters = t.refine_iters;
    A.out_depth = out_depth;
    A.out_normal = out_normal;
    A.wrec = static_cast<unsigned long long*>(s->d_wrec);
    hipError_t e = fill_u32(reinterpret_cast<uint32_t*>(s->d_stats), 2u * kStatCount, 0u, stream);
    if (e != hipSuccess) return device_error(e, "ablation: clear stats");
    if (variant == ST_ABLATION_FAST_PTR)
        hipLaunchKernelGGL(ablation_trace_kernel<true>, grid, dim3(64), 0, stream, A);
    else
        hipLaunchKernelGGL(ablation_trace_kernel<false>, grid, dim3(64), 0, stream, A);
    e = hipGetLastError();
    if (e != hipSuccess) return device_error(e, "ablation_trace_kernel");
    if (out_stats) {
        e = launch_reduce_counters(A.wrec, n_blocks, s->d_stats, stream);
        if (e != hipSuccess) return device_error(e, "ablation: counter reduction");
        unsigned long long h[kStatCount];
        e = hipMemcpyAsync(h, s->d_stats, sizeof(h), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return device_error(e, "ablation stats");
        stats_from_counters(s, h, out_stats);
        out_stats->abuffer_entries = s->n_dexels;
    }
    return ST_OK;
}
