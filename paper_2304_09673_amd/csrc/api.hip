// C ABI entry points (include/st.h): argument checking, device memory,
// camera set-up, and the calls into the host preprocessing, the A-buffer
// build and the tracer.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "st_internal.h"
#include "st_mlp.h"

namespace st {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

st_status device_error(hipError_t e, const char* where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return ST_E_DEVICE;
}

void* dev_alloc(st_scene* s, size_t bytes, hipStream_t stream) {
    if (bytes == 0) bytes = 256;
    if (s->has_alloc) return s->alloc.alloc(bytes, (void*)stream, s->alloc.ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(st_scene* s, void* p, hipStream_t stream) {
    if (!p) return;
    if (s->has_alloc) { s->alloc.free(p, (void*)stream, s->alloc.ctx); return; }
    (void)hipFree(p);
}

static void free_abuffer(st_scene* s, hipStream_t stream) {
    dev_free(s, s->d_tile_off, stream); s->d_tile_off = nullptr;
    dev_free(s, s->d_tile_ovl, stream); s->d_tile_ovl = nullptr;
    dev_free(s, s->d_tile_order, stream); s->d_tile_order = nullptr;
    dev_free(s, s->d_tile_cnt, stream); s->d_tile_cnt = nullptr;
    dev_free(s, s->d_e_node, stream); s->d_e_node = nullptr;
    dev_free(s, s->d_e_zin, stream); s->d_e_zin = nullptr;
    dev_free(s, s->d_e_zout, stream); s->d_e_zout = nullptr;
    dev_free(s, s->d_wide, stream); s->d_wide = nullptr;
    dev_free(s, s->d_scratch, stream); s->d_scratch = nullptr;
    dev_free(s, s->d_slots, stream); s->d_slots = nullptr;
    s->slots_bytes = 0;
    dev_free(s, s->d_wrec, stream); s->d_wrec = nullptr;
    dev_free(s, s->d_dx_meta, stream); s->d_dx_meta = nullptr;
    s->dx_meta_bytes = 0;
    dev_free(s, s->d_dx, stream); s->d_dx = nullptr;
    s->dx_bytes = 0;
    s->wrec_bytes = 0;
    s->scratch_bytes = 0;
    s->ab_cap = 0;
    s->n_tiles = 0;
    s->ab_valid = false;
}

static bool make_devcam(const st_camera& c, DevCam& d) {
    double fwd[3], up[3], right[3];
    for (int j = 0; j < 3; j++) {
        if (!std::isfinite(c.eye[j]) || !std::isfinite(c.target[j]) || !std::isfinite(c.up[j])) return false;
        fwd[j] = double(c.target[j]) - c.eye[j];
    }
    double fn = std::sqrt(fwd[0] * fwd[0] + fwd[1] * fwd[1] + fwd[2] * fwd[2]);
    if (!(fn > 0)) return false;
    for (int j = 0; j < 3; j++) fwd[j] /= fn;
    right[0] = fwd[1] * c.up[2] - fwd[2] * c.up[1];
    right[1] = fwd[2] * c.up[0] - fwd[0] * c.up[2];
    right[2] = fwd[0] * c.up[1] - fwd[1] * c.up[0];
    double rn = std::sqrt(right[0] * right[0] + right[1] * right[1] + right[2] * right[2]);
    if (!(rn > 1e-12)) return false;
    for (int j = 0; j < 3; j++) right[j] /= rn;
    up[0] = right[1] * fwd[2] - right[2] * fwd[1];
    up[1] = right[2] * fwd[0] - right[0] * fwd[2];
    up[2] = right[0] * fwd[1] - right[1] * fwd[0];
    double th = std::tan(0.5 * double(c.vfov_deg) * M_PI / 180.0);
    for (int j = 0; j < 3; j++) {
        d.eye[j] = c.eye[j];
        d.fwd[j] = float(fwd[j]);
        d.right[j] = float(right[j]);
        d.up[j] = float(up[j]);
    }
    d.tx = float(th * double(c.width) / double(c.height));
    d.ty = float(th);
    d.inv_w2 = float(2.0 / c.width);
    d.inv_h2 = float(2.0 / c.height);
    d.w = c.width;
    d.h = c.height;
    return true;
}

void stats_from_counters(const st_scene* s, const unsigned long long* h, st_stats* out) {
    std::memset(out, 0, sizeof(*out));
    out->rays = h[0];
    out->hits = h[1];
    out->unconverged = h[2];
    out->field_evals = h[3];
    out->grad_evals = h[4];
    for (int q = 0; q < 4; q++) {
        out->node_evals[q] = h[5 + q];
        out->grad_node_evals[q] = h[9 + q];
    }
    out->steps = h[13];
    out->subfrustums = h[14];
    out->empty_views = h[15];
    out->view_nodes = h[16];
    out->max_active = h[17];
    out->wide_tiles = h[18];
    out->learned_accepted = h[19];
    out->learned_rejected = h[20];
    out->stalled = h[21];
    out->smooth_evals = h[22];
    out->block_cycles_max = h[23];
    out->block_cycles_sum = h[24];
    out->abuffer_entries = uint64_t(s->n_live);
    out->abuffer_binned = uint64_t(s->n_entries);
    out->abuffer_candidates = uint64_t(s->n_cand);
    for (int k = 0; k < 3; k++) out->candidate_pixels[k] = s->cand_pix[k];
    out->abuffer_tested = uint64_t(s->n_tested);
    out->max_list = s->max_list;
    out->max_overlap = s->max_overlap;
}

static st_status check_tuning(const st_tuning& t) {
    if (t.tile != 8 && t.tile != 16 && t.tile != 32) { set_error("tuning: tile must be 8, 16 or 32"); return ST_E_INVALID; }
    if (t.max_active < 2) { set_error("tuning: max_active < 2"); return ST_E_INVALID; }
    if (!(t.sub_depth > 0.f) || !std::isfinite(t.sub_depth)) { set_error("tuning: sub_depth must be > 0"); return ST_E_INVALID; }
    if (t.max_new < 1) { set_error("tuning: max_new < 1"); return ST_E_INVALID; }
    if (!(t.eps > 0.f) || !std::isfinite(t.eps)) { set_error("tuning: eps must be > 0"); return ST_E_INVALID; }
    if (t.max_steps < 1 || t.refine_iters < 0 || t.refine_iters > 64) { set_error("tuning: step limits"); return ST_E_INVALID; }
    if (t.step_mode < ST_STEP_PLAIN || t.step_mode > ST_STEP_SEGMENT) { set_error("tuning: step_mode"); return ST_E_INVALID; }
    if (!(t.omega >= 1.f) || !(t.omega <= 4.f)) { set_error("tuning: omega outside [1, 4]"); return ST_E_INVALID; }
    if (!(t.lipschitz >= 0.f) || !std::isfinite(t.lipschitz)) { set_error("tuning: lipschitz < 0"); return ST_E_INVALID; }
    if (t.keep_all_entries != 0 && t.keep_all_entries != 1) { set_error("tuning: keep_all_entries must be 0 or 1"); return ST_E_INVALID; }
    if (!std::isfinite(t.probe_step)) { set_error("tuning: probe_step not finite"); return ST_E_INVALID; }
    return ST_OK;
}

}  // namespace st

using namespace st;

extern "C" {

const char* st_status_str(st_status s) {
    switch (s) {
    case ST_OK: return "ok";
    case ST_E_INVALID: return "invalid argument";
    case ST_E_TREE: return "malformed blobtree";
    case ST_E_CAPACITY: return "capacity exceeded";
    case ST_E_NOMEM: return "out of memory";
    case ST_E_DEVICE: return "device error";
    case ST_E_STALE: return "stale A-buffer";
    }
    return "unknown status";
}

const char* st_last_error(void) { return g_err.c_str(); }

st_status st_default_tuning(st_tuning* t) {
    if (!t) { set_error("NULL tuning"); return ST_E_INVALID; }
    std::memset(t, 0, sizeof(*t));
    t->tile = 16;
    t->max_active = 256;
    t->sub_depth = 1.0f / 20.0f;
    t->max_new = 6;
    t->eps = 1e-4f;
    t->max_steps = 1024;
    t->refine_iters = 8;
    t->step_mode = ST_STEP_PLAIN;
    t->omega = 1.7f;
    t->lipschitz = 0.f;
    t->probe_step = 1e-3f;
    return ST_OK;
}

st_status st_flatten_blobtree(const st_node* nodes, int32_t n, int32_t root, const st_allocator* alloc,
                              void* stream_v, st_scene** out) {
    if (!out) { set_error("flatten: NULL out"); return ST_E_INVALID; }
    *out = nullptr;
    hipStream_t stream = (hipStream_t)stream_v;
    st_scene* s = new (std::nothrow) st_scene();
    if (!s) { set_error("flatten: host allocation failed"); return ST_E_NOMEM; }
    if (alloc) {
        if (!alloc->alloc || !alloc->free) { delete s; set_error("flatten: allocator without alloc/free"); return ST_E_INVALID; }
        s->alloc = *alloc;
        s->has_alloc = true;
    }
    st_status r;
    try {
        r = flatten_host(nodes, n, root, s);
    } catch (const std::bad_alloc&) {
        r = ST_E_NOMEM;
        set_error("flatten: host allocation failed");
    }
    if (r != ST_OK) { delete s; return r; }
    size_t N = size_t(s->n_nodes), P = size_t(s->n_prims);
    struct { void** p; size_t bytes; const void* src; } bufs[] = {
        {(void**)&s->d_blob, N * 4, s->h_blob.data()},
        {(void**)&s->d_kill, N * 4, s->h_kill.data()},
        {(void**)&s->d_kslot, N * 32, s->h_kslot.data()},
        {(void**)&s->d_rmq, s->h_rmq.size() * 4, s->h_rmq.data()},
        {(void**)&s->d_prims, P * 4, s->h_prims.data()},
        {(void**)&s->d_sub, N * 32, s->h_sub.data()},
        {(void**)&s->d_oside, P * 32, s->h_oside.data()},
        {(void**)&s->d_fast, N * 4, s->h_fast.data()},
        {(void**)&s->d_pslot, N * 4, s->h_pslot.data()},
        {(void**)&s->d_par, N * sizeof(NodePar), s->h_par.data()},
        {(void**)&s->d_roi, N * 4, s->h_roi.data()},
        {(void**)&s->d_voi, P * sizeof(Voi), nullptr},
        {(void**)&s->d_stats, kStatCount * 8, nullptr},
        {(void**)&s->d_misc, 64 * 4, nullptr},
    };
    for (auto& b : bufs) {
        *b.p = dev_alloc(s, b.bytes, stream);
        if (!*b.p) { st_scene_destroy(s); set_error("flatten: device allocation failed"); return ST_E_NOMEM; }
        s->device_bytes += b.bytes;
        if (b.src) {
            hipError_t e = hipMemcpyAsync(*b.p, b.src, b.bytes, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) { st_scene_destroy(s); return device_error(e, "flatten upload"); }
        }
    }
    r = launch_voi(s, stream);
    if (r != ST_OK) { st_scene_destroy(s); return r; }
    hipError_t e = hipStreamSynchronize(stream);   // host arrays stay owned by the scene; keep the copy simple
    if (e != hipSuccess) { st_scene_destroy(s); return device_error(e, "flatten sync"); }
    *out = s;
    return ST_OK;
}

void st_scene_destroy(st_scene* s) {
    if (!s) return;
    hipStream_t stream = nullptr;
    for (hipEvent_t ev : s->test_events) (void)hipEventDestroy(ev);
    free_abuffer(s, stream);
    dev_free(s, s->d_blob, stream);
    dev_free(s, s->d_kill, stream);
    dev_free(s, s->d_kslot, stream);
    dev_free(s, s->d_rmq, stream);
    dev_free(s, s->d_prims, stream);
    dev_free(s, s->d_sub, stream);
    dev_free(s, s->d_oside, stream);
    dev_free(s, s->d_fast, stream);
    dev_free(s, s->d_pslot, stream);
    dev_free(s, s->d_par, stream);
    dev_free(s, s->d_roi, stream);
    dev_free(s, s->d_voi, stream);
    dev_free(s, s->d_stats, stream);
    dev_free(s, s->d_misc, stream);
    dev_free(s, s->d_mlp, stream);
    dev_free(s, s->d_long, stream);
    delete s;
}

st_status st_scene_get_info(const st_scene* s, st_scene_info* info) {
    if (!s || !info) { set_error("info: NULL argument"); return ST_E_INVALID; }
    info->n_nodes = s->n_nodes;
    info->n_prims = s->n_prims;
    info->depth = s->depth;
    info->extent = s->extent;
    info->lipschitz = s->lipschitz;
    for (int j = 0; j < 3; j++) { info->voi_lo[j] = s->voi_lo[j]; info->voi_hi[j] = s->voi_hi[j]; }
    info->device_bytes = s->device_bytes;
    info->abuffer_bytes = uint64_t(s->ab_cap) * 12 + uint64_t(s->n_tiles + 1) * 8;
    return ST_OK;
}

st_status st_update_primitives(st_scene* s, const int32_t* ids, const st_node* nodes, int32_t n, void* stream_v) {
    if (!s || n < 0 || (n > 0 && (!ids || !nodes))) { set_error("update: bad argument"); return ST_E_INVALID; }
    if (n == 0) return ST_OK;
    hipStream_t stream = (hipStream_t)stream_v;
    // validate everything before touching the scene
    std::vector<int32_t> slot(static_cast<size_t>(n));
    for (int i = 0; i < n; i++) {
        int32_t c = ids[i];
        if (c < 0 || c >= s->n_nodes) { set_error("update: node index out of range"); return ST_E_INVALID; }
        int32_t p = s->post_of_caller[size_t(c)];
        if (!blob_prim(s->h_blob[size_t(p)])) { set_error("update: node is not a primitive"); return ST_E_INVALID; }
        if (nodes[i].kind != blob_op(s->h_blob[size_t(p)])) { set_error("update: primitive kind changed"); return ST_E_INVALID; }
        st_status r = validate_primitive(nodes[i], c);
        if (r != ST_OK) return r;
        auto it = std::lower_bound(s->h_prims.begin(), s->h_prims.end(), uint32_t(p));
        slot[size_t(i)] = int32_t(it - s->h_prims.begin());
    }
    for (int i = 0; i < n; i++) {
        int32_t p = s->post_of_caller[size_t(ids[i])];
        primitive_params(nodes[i], double(s->h_roi[size_t(p)]), s->h_par[size_t(p)], s->h_box[size_t(slot[size_t(i)])]);
    }
    scene_bounds(s);
    subtree_boxes(s);
    hipError_t e = hipMemcpyAsync(s->d_sub, s->h_sub.data(), s->h_sub.size() * 4, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return device_error(e, "update: upload");
    if (n <= 64) {
        for (int i = 0; i < n && e == hipSuccess; i++) {
            size_t p = size_t(s->post_of_caller[size_t(ids[i])]);
            e = hipMemcpyAsync(s->d_par + p, &s->h_par[p], sizeof(NodePar), hipMemcpyHostToDevice, stream);
        }
    } else {
        e = hipMemcpyAsync(s->d_par, s->h_par.data(), s->h_par.size() * sizeof(NodePar), hipMemcpyHostToDevice, stream);
    }
    if (e != hipSuccess) return device_error(e, "update: upload");
    st_status r = launch_voi(s, stream);
    if (r != ST_OK) return r;
    // the host copies are read by the asynchronous uploads
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_error(e, "update: sync");
    s->ab_valid = false;   // the A-buffer must be rebuilt
    return ST_OK;
}

st_status st_build_abuffer(st_scene* s, const st_camera* cam, const st_tuning* tin, void* stream_v) {
    if (!s || !cam) { set_error("build: NULL argument"); return ST_E_INVALID; }
    hipStream_t stream = (hipStream_t)stream_v;
    st_tuning t;
    if (tin) t = *tin; else st_default_tuning(&t);
    st_status r = check_tuning(t);
    if (r != ST_OK) return r;
    if (cam->width <= 0 || cam->height <= 0 || !(cam->vfov_deg > 0.f) || !(cam->vfov_deg < 180.f)) {
        set_error("build: camera size <= 0 or field of view outside (0, 180)");
        return ST_E_INVALID;
    }
    if (int64_t(cam->width) * cam->height > (int64_t(1) << 30)) { set_error("build: image too large"); return ST_E_CAPACITY; }
    DevCam dc;
    if (!make_devcam(*cam, dc)) { set_error("build: degenerate camera basis"); return ST_E_INVALID; }
    int tx = (cam->width + t.tile - 1) / t.tile, ty = (cam->height + t.tile - 1) / t.tile;
    int T = tx * ty;
    // Same scene, camera and tuning as the valid A-buffer: every count and
    // size of the build is the same, so it is rerun on the device with the
    // sizes of the last one (no host synchronization, no allocation).
    if (s->ab_valid && T == s->n_tiles && std::memcmp(cam, &s->ab_cam, sizeof(st_camera)) == 0 &&
        std::memcmp(&t, &s->ab_tune, sizeof(st_tuning)) == 0) {
        r = build_abuffer_device(s, t, stream, true);
        if (r != ST_OK) { s->ab_valid = false; return r; }
        s->ab_gen++;
        return ST_OK;
    }
    if (T != s->n_tiles || !s->d_tile_off) {
        dev_free(s, s->d_tile_off, stream);
        dev_free(s, s->d_tile_ovl, stream);
        dev_free(s, s->d_tile_order, stream);
        dev_free(s, s->d_tile_cnt, stream);
        dev_free(s, s->d_wide, stream);
        s->d_tile_off = (uint32_t*)dev_alloc(s, size_t(T + 1) * 4, stream);
        s->d_tile_ovl = (uint32_t*)dev_alloc(s, size_t(T) * 4, stream);
        s->d_tile_order = (uint32_t*)dev_alloc(s, size_t(T) * 4, stream);
        s->d_tile_cnt = (uint32_t*)dev_alloc(s, size_t(T) * 4, stream);
        s->d_wide = (uint32_t*)dev_alloc(s, size_t(T + 1) * 4, stream);
        if (!s->d_tile_off || !s->d_tile_ovl || !s->d_tile_order || !s->d_tile_cnt || !s->d_wide) {
            set_error("build: tile arrays allocation failed");
            return ST_E_NOMEM;
        }
    }
    s->dcam = dc;
    s->tiles_x = tx;
    s->tiles_y = ty;
    s->n_tiles = T;
    // view-depth span of the box of all volumes of interest
    double zmin = INFINITY, zmax = -INFINITY;
    for (int c = 0; c < 8; c++) {
        double p[3] = {(c & 1) ? s->voi_hi[0] : s->voi_lo[0], (c & 2) ? s->voi_hi[1] : s->voi_lo[1],
                       (c & 4) ? s->voi_hi[2] : s->voi_lo[2]};
        double z = 0;
        for (int j = 0; j < 3; j++) z += (p[j] - cam->eye[j]) * dc.fwd[j];
        zmin = std::min(zmin, z);
        zmax = std::max(zmax, z);
    }
    s->z_min = float(std::max(zmin, 0.0));
    s->z_max = float(std::max(zmax, 0.0));
    s->ab_ma_fast = std::min(t.max_active, 256);
    s->ab_ma_wide = 1024;
    s->ab_valid = false;
    r = build_abuffer_device(s, t, stream);
    if (r != ST_OK) return r;
    s->ab_cam = *cam;
    s->ab_tune = t;
    s->ab_valid = true;
    s->ab_gen++;
    return ST_OK;
}

st_status st_trace(st_scene* s, const st_camera* cam, float* out_depth, float* out_normal, st_stats* out_stats,
                   void* stream_v) {
    return st_trace_ex(s, cam, out_depth, out_normal, nullptr, out_stats, stream_v);
}

st_status st_trace_ex(st_scene* s, const st_camera* cam, float* out_depth, float* out_normal, uint32_t* out_info,
                      st_stats* out_stats, void* stream_v) {
    if (!s || !cam || !out_depth || !out_normal) { set_error("trace: NULL argument"); return ST_E_INVALID; }
    hipStream_t stream = (hipStream_t)stream_v;
    if (!s->ab_valid || std::memcmp(cam, &s->ab_cam, sizeof(st_camera)) != 0) {
        set_error("trace: the A-buffer was not built for this camera");
        return ST_E_STALE;
    }
    st_status r = trace_device(s, s->ab_tune, out_depth, out_normal, out_info, stream, nullptr, out_stats != nullptr);
    if (r != ST_OK) return r;
    if (out_stats) {
        unsigned long long h[kStatCount];
        hipError_t e = hipMemcpyAsync(h, s->d_stats, sizeof(h), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return device_error(e, "trace stats");
        stats_from_counters(s, h, out_stats);
    }
    return ST_OK;
}

static st_status active_to_post(const st_scene* s, const int32_t* active, int32_t n_active,
                                std::vector<uint32_t>& post) {
    post.clear();
    if (!active) {
        post.assign(s->h_prims.begin(), s->h_prims.end());
        return ST_OK;
    }
    if (n_active < 0) { set_error("n_active < 0"); return ST_E_INVALID; }
    for (int i = 0; i < n_active; i++) {
        int32_t c = active[i];
        if (c < 0 || c >= s->n_nodes) { set_error("active index out of range"); return ST_E_INVALID; }
        int32_t p = s->post_of_caller[size_t(c)];
        if (!blob_prim(s->h_blob[size_t(p)])) { set_error("active node is not a primitive"); return ST_E_INVALID; }
        post.push_back(uint32_t(p));
    }
    std::sort(post.begin(), post.end());
    if (std::adjacent_find(post.begin(), post.end()) != post.end()) { set_error("duplicate active primitive"); return ST_E_INVALID; }
    return ST_OK;
}

st_status st_autotune(st_scene* s, const st_camera* cam, const st_tuning* base, int32_t reps, st_tuning* out,
                      float* out_ms, void* stream_v) {
    if (!s || !cam || !out || reps < 1) { set_error("autotune: NULL argument or reps < 1"); return ST_E_INVALID; }
    hipStream_t stream = (hipStream_t)stream_v;
    st_tuning b;
    if (base) b = *base; else st_default_tuning(&b);
    size_t pix = size_t(cam->width > 0 ? cam->width : 0) * size_t(cam->height > 0 ? cam->height : 0);
    float* buf = (float*)dev_alloc(s, pix * 16 + 256, stream);
    if (!buf) { set_error("autotune: output buffer allocation failed"); return ST_E_NOMEM; }
    float* depth = buf;
    float* normal = buf + pix;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) { dev_free(s, buf, stream); return device_error(he, "autotune events"); }
    const int tiles[3] = {8, 16, 32};
    const int news[4] = {6, 16, 64, 256};
    const float subs[2] = {1.0f / 20.0f, 0.25f};
    float best = INFINITY;
    st_tuning best_t = b;
    st_status r = ST_OK;
    for (int ti = 0; ti < 3 && r == ST_OK; ti++)
        for (int ni = 0; ni < 4 && r == ST_OK; ni++)
            for (int si = 0; si < 2 && r == ST_OK; si++) {
                st_tuning t = b;
                t.tile = tiles[ti];
                t.max_new = news[ni];
                t.sub_depth = subs[si];
                std::vector<float> ms;
                for (int k = 0; k <= reps && r == ST_OK; k++) {   // first run warms up
                    he = hipEventRecord(e0, stream);
                    if (he != hipSuccess) { r = device_error(he, "autotune record"); break; }
                    r = st_build_abuffer(s, cam, &t, stream_v);
                    if (r != ST_OK) break;
                    r = trace_device(s, s->ab_tune, depth, normal, nullptr, stream);
                    if (r != ST_OK) break;
                    he = hipEventRecord(e1, stream);
                    if (he == hipSuccess) he = hipEventSynchronize(e1);
                    float dt = 0.f;
                    if (he == hipSuccess) he = hipEventElapsedTime(&dt, e0, e1);
                    if (he != hipSuccess) { r = device_error(he, "autotune timing"); break; }
                    if (k > 0) ms.push_back(dt);
                }
                if (r != ST_OK) break;
                std::sort(ms.begin(), ms.end());
                float med = ms[ms.size() / 2];
                if (med < best) { best = med; best_t = t; }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dev_free(s, buf, stream);
    if (r != ST_OK) return r;
    r = st_build_abuffer(s, cam, &best_t, stream_v);
    if (r != ST_OK) return r;
    *out = best_t;
    if (out_ms) *out_ms = best;
    return ST_OK;
}

st_status st_debug_prune_tree(const st_node* nodes, int32_t n, int32_t root, const int32_t* active,
                              int32_t n_active, int32_t* out_nodes, int32_t cap, int32_t* out_len, float* out_lip) {
    if (!out_len) { set_error("prune: NULL out_len"); return ST_E_INVALID; }
    st_scene s;
    st_status r;
    try {
        r = flatten_host(nodes, n, root, &s);
        if (r != ST_OK) return r;
        std::vector<uint32_t> post, view;
        r = active_to_post(&s, active, n_active, post);
        if (r != ST_OK) return r;
        PruneResult pr = host_prune(&s, post, view);
        *out_len = pr.len;
        if (out_lip) *out_lip = pr.lip;
        if (pr.len > 0) {
            if (!out_nodes || cap < pr.len) { set_error("prune: output capacity too small"); return ST_E_CAPACITY; }
            for (int i = 0; i < pr.len; i++) out_nodes[i] = s.caller_of_post[ventry_node(view[size_t(i)])];
        }
    } catch (const std::bad_alloc&) {
        set_error("prune: host allocation failed");
        return ST_E_NOMEM;
    }
    return ST_OK;
}

st_status st_debug_sparse_traversal(const st_node* nodes, int32_t n, int32_t root, const int32_t* active,
                                    int32_t n_active, int32_t variant, int32_t* out_nodes, int32_t cap,
                                    int32_t* out_len, float* out_lip, int32_t* out_visited) {
    if (!out_len) { set_error("sparse: NULL out_len"); return ST_E_INVALID; }
    if (variant != ST_ABLATION_PARENT_PTR && variant != ST_ABLATION_FAST_PTR) {
        set_error("sparse: variant must be ST_ABLATION_PARENT_PTR or ST_ABLATION_FAST_PTR");
        return ST_E_INVALID;
    }
    st_scene s;
    try {
        st_status r = flatten_host(nodes, n, root, &s);
        if (r != ST_OK) return r;
        std::vector<uint32_t> post, view;
        r = active_to_post(&s, active, n_active, post);
        if (r != ST_OK) return r;
        float lip = 0.f;
        uint32_t visited = 0;
        r = host_sparse(&s, post, variant == ST_ABLATION_FAST_PTR, view, lip, visited);
        if (r != ST_OK) return r;
        *out_len = int32_t(view.size());
        if (out_lip) *out_lip = lip;
        if (out_visited) *out_visited = int32_t(visited);
        if (!view.empty()) {
            if (!out_nodes || cap < int32_t(view.size())) { set_error("sparse: output capacity too small"); return ST_E_CAPACITY; }
            for (size_t i = 0; i < view.size(); i++) out_nodes[i] = s.caller_of_post[view[i]];
        }
    } catch (const std::bad_alloc&) {
        set_error("sparse: host allocation failed");
        return ST_E_NOMEM;
    }
    return ST_OK;
}

st_status st_debug_eval_field(const st_scene* s, const int32_t* active, int32_t n_active, const float* pts,
                              int32_t n_pts, float* out_f, float* out_grad, int32_t* out_root_used,
                              int32_t* out_view, int32_t view_cap, int32_t* out_view_len, void* stream_v) {
    if (!s || (n_pts > 0 && (!pts || !out_f)) || n_pts < 0) { set_error("eval: NULL argument"); return ST_E_INVALID; }
    hipStream_t stream = (hipStream_t)stream_v;
    std::vector<uint32_t> post;
    st_status r = active_to_post(s, active, n_active, post);
    if (r != ST_OK) return r;
    int n = int(post.size());
    if (n > 1024) { set_error("eval: active set larger than the largest view"); return ST_E_CAPACITY; }
    // device buffer: sorted active list + [used, len, lip, pad] + view copy
    size_t bytes = size_t(n) * 4 + 256 + 16 + 2048 * 4 + 256;
    st_scene* sm = const_cast<st_scene*>(s);
    char* buf = (char*)dev_alloc(sm, bytes, stream);
    if (!buf) { set_error("eval: allocation failed"); return ST_E_NOMEM; }
    uint32_t* d_act = (uint32_t*)buf;
    int* d_ru = (int*)(buf + ((size_t(n) * 4 + 255) & ~size_t(255)));
    hipError_t e = hipSuccess;
    if (n > 0) e = hipMemcpyAsync(d_act, post.data(), size_t(n) * 4, hipMemcpyHostToDevice, stream);
    int hdr[4] = {0, 0, 0, 0};
    std::vector<uint32_t> hview(2048, 0u);
    if (e == hipSuccess && n > 0) {
        r = debug_eval_device(s, d_act, n, pts, n_pts, out_f, out_grad, d_ru, stream);
        if (r != ST_OK) { dev_free(sm, buf, stream); return r; }
        e = hipMemcpyAsync(hdr, d_ru, 16, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(hview.data(), d_ru + 4, 2048 * 4, hipMemcpyDeviceToHost, stream);
    } else if (e == hipSuccess && n_pts > 0) {
        // empty active set: the pruned root is unused, f_A = +inf
        std::vector<float> inf(size_t(n_pts), INFINITY);
        e = hipMemcpyAsync(out_f, inf.data(), size_t(n_pts) * 4, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && out_grad) e = hipMemsetAsync(out_grad, 0, size_t(n_pts) * 12, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    dev_free(sm, buf, stream);
    if (e != hipSuccess) return device_error(e, "eval");
    if (out_root_used) *out_root_used = hdr[0];
    int vlen = hdr[0] ? hdr[1] : 0;
    if (out_view_len) *out_view_len = vlen;
    if (out_view) {
        if (view_cap < vlen) { set_error("eval: view capacity too small"); return ST_E_CAPACITY; }
        for (int i = 0; i < vlen; i++) out_view[i] = s->caller_of_post[ventry_node(hview[size_t(i)])];
    }
    return ST_OK;
}

st_status st_debug_kernel_timing(st_scene* s, int32_t enable, float* total_ms, int32_t* launches) {
    if (!s) { set_error("kernel timing: NULL scene"); return ST_E_INVALID; }
    if (enable) {
        s->time_test = true;
        s->test_used = 0;
        return ST_OK;
    }
    if (!total_ms || !launches) { set_error("kernel timing: NULL output"); return ST_E_INVALID; }
    s->time_test = false;
    float sum = 0.f;
    for (size_t k = 0; k < s->test_used; k++) {
        hipError_t e = hipEventSynchronize(s->test_events[2 * k + 1]);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, s->test_events[2 * k], s->test_events[2 * k + 1]);
        if (e != hipSuccess) return device_error(e, "kernel timing");
        sum += ms;
    }
    *total_ms = sum;
    *launches = int32_t(s->test_used);
    s->test_used = 0;
    return ST_OK;
}

st_status st_debug_abuffer(const st_scene* s, uint32_t* tile_off, size_t tile_cap, uint32_t* entries,
                           size_t entry_cap, int32_t* n_tiles, int64_t* n_entries, void* stream_v) {
    if (!s) { set_error("abuffer: NULL scene"); return ST_E_INVALID; }
    if (!s->ab_valid) { set_error("abuffer: not built"); return ST_E_STALE; }
    hipStream_t stream = (hipStream_t)stream_v;
    if (n_tiles) *n_tiles = s->n_tiles;
    if (n_entries) *n_entries = s->n_live;
    if (!tile_off && !entries) return ST_OK;
    if (tile_off && tile_cap < size_t(s->n_tiles + 1)) { set_error("abuffer: tile capacity"); return ST_E_CAPACITY; }
    if (entries && entry_cap < 3 * size_t(s->n_live)) { set_error("abuffer: entry capacity"); return ST_E_CAPACITY; }
    // the kept segment of every tile: [tile_off[t], tile_off[t] + tile_cnt[t])
    const size_t T = size_t(s->n_tiles), E = size_t(s->n_cand);
    std::vector<uint32_t> off(T + 1), cnt(T), a(E), b(E), c(E);
    hipError_t e = hipMemcpyAsync(off.data(), s->d_tile_off, (T + 1) * 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(cnt.data(), s->d_tile_cnt, T * 4, hipMemcpyDeviceToHost, stream);
    if (E && entries) {
        if (e == hipSuccess) e = hipMemcpyAsync(a.data(), s->d_e_node, E * 4, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(b.data(), s->d_e_zin, E * 4, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(c.data(), s->d_e_zout, E * 4, hipMemcpyDeviceToHost, stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess) {
        size_t k = 0;
        for (size_t t = 0; t < T; t++) {
            if (tile_off) tile_off[t] = uint32_t(k);
            for (uint32_t i = off[t]; i < off[t] + cnt[t] && i < E; i++, k++) {
                if (!entries) continue;
                entries[3 * k] = uint32_t(s->caller_of_post[a[i]]);
                entries[3 * k + 1] = b[i];
                entries[3 * k + 2] = c[i];
            }
        }
        if (tile_off) tile_off[T] = uint32_t(k);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_error(e, "abuffer copy");
    return ST_OK;
}

st_status st_set_step_model(st_scene* s, const float* weights, const float* norm, void* stream_v) {
    if (!s || !weights || !norm) { set_error("set_step_model: NULL argument"); return ST_E_INVALID; }
    hipStream_t stream = (hipStream_t)stream_v;
    if (!s->d_mlp) {
        s->d_mlp = (uint32_t*)dev_alloc(s, size_t(kMlpTabWords) * 4, stream);
        if (!s->d_mlp) { set_error("set_step_model: allocation failed"); return ST_E_NOMEM; }
    }
    st_status r = st_mlp_pack(weights, norm, s->d_mlp, stream);
    if (r == ST_OK) s->has_model = true;
    return r;
}

st_status st_trace_dump(st_scene* s, const st_camera* cam, float* out_depth, float* out_normal, float* features,
                        float* targets, int64_t cap, int64_t* n_samples, void* stream_v) {
    if (!s || !cam || !out_depth || !out_normal || !n_samples || cap < 0 || (cap > 0 && (!features || !targets))) {
        set_error("trace_dump: bad argument");
        return ST_E_INVALID;
    }
    hipStream_t stream = (hipStream_t)stream_v;
    if (!s->ab_valid || std::memcmp(cam, &s->ab_cam, sizeof(st_camera)) != 0) {
        set_error("trace_dump: the A-buffer was not built for this camera");
        return ST_E_STALE;
    }
    // the sample counter is the last stats word, cleared here (a fill
    // kernel, no memset)
    DumpTarget d{features, targets, s->d_stats + (kStatCount - 1), (unsigned long long)cap};
    hipError_t ec = fill_u32(reinterpret_cast<uint32_t*>(s->d_stats + (kStatCount - 1)), 2u, 0u, stream);
    if (ec != hipSuccess) return device_error(ec, "trace_dump: clear the sample counter");
    st_status r = trace_device(s, s->ab_tune, out_depth, out_normal, nullptr, stream, &d);
    if (r != ST_OK) return r;
    unsigned long long h = 0;
    hipError_t e = hipMemcpyAsync(&h, s->d_stats + (kStatCount - 1), 8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_error(e, "trace_dump count");
    *n_samples = int64_t(h);
    return ST_OK;
}

}  // extern "C"
