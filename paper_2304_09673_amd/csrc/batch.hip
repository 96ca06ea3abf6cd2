// Batched rendering of many scenes from one work queue (not in the paper).
//
// A frame of the batch is: for every scene, the A-buffer build replayed with
// the sizes of its first build (no host synchronization, no allocation), then
// two persistent kernels that pull (scene, tile, 8x8 block) jobs from global
// atomic queues, longest tile list first: one for blocks whose tiles fit the
// LDS capacity of the fast path, one for the rest (wide capacity).  The whole
// frame is captured once into a HIP graph and replayed with one launch.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "st_trace.h"

namespace st {

// Batched rendering is switched off: its creation (first builds, one direct
// frame, graph capture) did not return on the device, and the cause has not
// been found.  Every entry point refuses with ST_E_INVALID until it is.
constexpr bool kBatchEnabled = false;

// Next job index of the wave from the global queue.  Every lane takes part
// in the atomic (lane 0 adds 1, the others 0) and the index is lane 0's
// return value, so the fetch has no lane-dependent branch: a persistent loop
// whose job index is produced under a lane-0-only branch was compiled into a
// loop that can re-enter its body with the index register reset to 0.
__device__ __forceinline__ uint32_t next_job(uint32_t* head) {
    const uint32_t r = atomicAdd(head, lane_id() == 0 ? 1u : 0u);
    return rdlane(r, 0);
}

// job: x = scene index, y = tile << 8 | block within the tile
template <int KS>
__global__ void __launch_bounds__(256) batch_fast_kernel(const TraceArgs* __restrict__ args,
                                                         const uint2* __restrict__ jobs, uint32_t n_jobs,
                                                         uint32_t* __restrict__ head) {
    __shared__ WaveLds<kMaFast> lds[4];
    const int w = int(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));   // wave-uniform: the LDS slot address stays scalar
    // a wave takes at most n_jobs jobs, so the loop ends even if the queue
    // were corrupted
    for (uint32_t it = 0; it < n_jobs; it++) {
        const uint32_t j = next_job(head);
        if (j >= n_jobs) break;
        const uint2 jb = jobs[j];
        const TraceArgs& A = args[jb.x];
        trace_block<WaveLds<kMaFast>, KS, SM_PLAIN>(A, lds[w], jb.y >> 8, jb.y & 255u, A.stats, nullptr);
    }
}

template <int KS, bool InLds>
__global__ void __launch_bounds__(64) batch_wide_kernel(const TraceArgs* __restrict__ args,
                                                        const uint2* __restrict__ jobs, uint32_t n_jobs,
                                                        uint32_t* __restrict__ head, uint32_t* slots, int ma) {
    extern __shared__ uint32_t dyn_slot[];
    WaveGlob S{InLds ? dyn_slot : slots + size_t(blockIdx.x) * slot_words(ma), ma};
    for (uint32_t it = 0; it < n_jobs; it++) {
        const uint32_t j = next_job(head);
        if (j >= n_jobs) break;
        const uint2 jb = jobs[j];
        const TraceArgs& A = args[jb.x];
        trace_block<WaveGlob, KS, SM_PLAIN>(A, S, jb.y >> 8, jb.y & 255u, A.stats, nullptr);
    }
}

}  // namespace st

using namespace st;

struct st_batch {
    std::vector<st_scene*> scenes;
    std::vector<uint64_t> gens;
    st_tuning tune{};
    st_scene* owner = nullptr;        // allocator of the batch's own buffers: the first scene
    TraceArgs* d_args = nullptr;
    uint2* d_jobs = nullptr;          // fast jobs, then wide jobs
    uint32_t n_fast = 0, n_wide = 0;
    uint32_t* d_heads = nullptr;      // [0] fast queue, [1] wide queue
    uint32_t* d_slots = nullptr;      // wide path in global memory (slots above the LDS size)
    int ma = 0;
    bool deep = false;                // evaluation stack 32 (some tree deeper than 16)
    uint32_t grid_fast = 0, grid_wide = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

st_status enqueue_frame(st_batch* b, hipStream_t stream) {
    hipError_t e;
    for (st_scene* s : b->scenes) {
        st_status r = build_abuffer_device(s, b->tune, stream, true);
        if (r != ST_OK) return r;
        e = fill_u32(reinterpret_cast<uint32_t*>(s->d_stats), 2u * kStatCount, 0u, stream);
        if (e != hipSuccess) return device_error(e, "batch: clear stats");
    }
    e = fill_u32(b->d_heads, 2u, 0u, stream);
    if (e != hipSuccess) return device_error(e, "batch: clear queues");
    if (b->n_fast) {
        if (b->deep)
            hipLaunchKernelGGL(batch_fast_kernel<32>, dim3(b->grid_fast), dim3(256), 0, stream, b->d_args, b->d_jobs,
                               b->n_fast, b->d_heads);
        else
            hipLaunchKernelGGL(batch_fast_kernel<16>, dim3(b->grid_fast), dim3(256), 0, stream, b->d_args, b->d_jobs,
                               b->n_fast, b->d_heads);
        e = hipGetLastError();
        if (e != hipSuccess) return device_error(e, "batch_fast_kernel");
    }
    if (b->n_wide) {
        const uint2* wj = b->d_jobs + b->n_fast;
        if (slot_words(b->ma) * 4u <= kSlotLdsBytes) {
            size_t shm = slot_words(b->ma) * 4u;
            if (b->deep)
                hipLaunchKernelGGL((batch_wide_kernel<32, true>), dim3(b->grid_wide), dim3(64), shm, stream, b->d_args,
                                   wj, b->n_wide, b->d_heads + 1, b->d_slots, b->ma);
            else
                hipLaunchKernelGGL((batch_wide_kernel<16, true>), dim3(b->grid_wide), dim3(64), shm, stream, b->d_args,
                                   wj, b->n_wide, b->d_heads + 1, b->d_slots, b->ma);
        } else {
            if (b->deep)
                hipLaunchKernelGGL((batch_wide_kernel<32, false>), dim3(b->grid_wide), dim3(64), 0, stream, b->d_args,
                                   wj, b->n_wide, b->d_heads + 1, b->d_slots, b->ma);
            else
                hipLaunchKernelGGL((batch_wide_kernel<16, false>), dim3(b->grid_wide), dim3(64), 0, stream, b->d_args,
                                   wj, b->n_wide, b->d_heads + 1, b->d_slots, b->ma);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return device_error(e, "batch_wide_kernel");
    }
    return ST_OK;
}

void batch_free(st_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->owner) {
        dev_free(b->owner, b->d_args, nullptr);
        dev_free(b->owner, b->d_jobs, nullptr);
        dev_free(b->owner, b->d_heads, nullptr);
        dev_free(b->owner, b->d_slots, nullptr);
    }
    delete b;
}

}  // namespace

extern "C" {

st_status st_batch_create(st_scene* const* scenes, const st_camera* cams, int32_t n, const st_tuning* tuning,
                          float* const* depths, float* const* normals, void* stream_v, st_batch** out) {
    if (!scenes || !cams || !depths || !normals || !out || n <= 0) {
        set_error("batch: bad argument");
        return ST_E_INVALID;
    }
    *out = nullptr;
    if (!kBatchEnabled) {
        set_error("batch: disabled (a batch creation did not return on the device and its cause is not "
                  "identified); render the scenes one by one with st_trace");
        return ST_E_INVALID;
    }
    hipStream_t stream = (hipStream_t)stream_v;
    st_tuning t;
    if (tuning) t = *tuning; else st_default_tuning(&t);
    if (t.step_mode != ST_STEP_PLAIN) { set_error("batch: only the plain step mode is batched"); return ST_E_INVALID; }
    for (int i = 0; i < n; i++) {
        if (!scenes[i] || !depths[i] || !normals[i]) { set_error("batch: NULL scene or output"); return ST_E_INVALID; }
        for (int j = 0; j < i; j++)
            if (scenes[j] == scenes[i]) { set_error("batch: a scene appears twice"); return ST_E_INVALID; }
    }
    st_batch* b = new (std::nothrow) st_batch;
    if (!b) { set_error("batch: out of host memory"); return ST_E_NOMEM; }
    b->tune = t;
    b->owner = scenes[0];
    std::vector<TraceArgs> args(static_cast<size_t>(n));
    struct Job { uint32_t len; uint32_t scene; uint32_t code; bool wide; };
    std::vector<Job> jobs;
    const uint32_t spt = uint32_t((t.tile / 8) * (t.tile / 8));
    int ma = 0;
    for (int i = 0; i < n; i++) {
        st_scene* s = scenes[i];
        // first build: sizes every buffer (synchronizes)
        st_status r = st_build_abuffer(s, &cams[i], &t, stream);
        if (r != ST_OK) { batch_free(b); return r; }
        b->scenes.push_back(s);
        b->gens.push_back(s->ab_gen);
        b->deep = b->deep || s->depth > 16;
        fill_trace_args(s, t, depths[i], normals[i], nullptr, args[size_t(i)]);
        std::vector<uint32_t> cnt(size_t(s->n_tiles)), ovl(size_t(s->n_tiles));
        hipError_t e = hipMemcpyAsync(cnt.data(), s->d_tile_cnt, cnt.size() * 4, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(ovl.data(), s->d_tile_ovl, ovl.size() * 4, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) { batch_free(b); return device_error(e, "batch: tile sizes"); }
        bool any_wide = false;
        for (int tile = 0; tile < s->n_tiles; tile++) {
            bool wide = ovl[size_t(tile)] > uint32_t(s->ab_ma_fast);
            any_wide = any_wide || wide;
            for (uint32_t k = 0; k < spt; k++)
                jobs.push_back({cnt[size_t(tile)], uint32_t(i), (uint32_t(tile) << 8) | k, wide});
        }
        if (any_wide) ma = std::max(ma, wide_capacity(s));
    }
    // longest tile list first, fast jobs then wide jobs
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& c) {
        if (a.wide != c.wide) return !a.wide;
        return a.len > c.len;
    });
    std::vector<uint2> hj(jobs.size());
    for (size_t k = 0; k < jobs.size(); k++) {
        hj[k] = make_uint2(jobs[k].scene, jobs[k].code);
        if (jobs[k].wide) b->n_wide++; else b->n_fast++;
    }
    if (jobs.size() >= (size_t(1) << 31)) { batch_free(b); set_error("batch: too many jobs"); return ST_E_CAPACITY; }
    b->ma = ma;
    // persistent grids: enough workgroups to fill the chip, never more than the jobs
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b->grid_fast = std::max(1u, std::min((b->n_fast + 3) / 4, uint32_t(cus) * 3u));
    b->grid_wide = b->n_wide ? std::min(b->n_wide, uint32_t(cus) * (ma <= 1024 ? 4u : 2u)) : 0u;
    b->d_args = (TraceArgs*)dev_alloc(b->owner, sizeof(TraceArgs) * size_t(n), stream);
    b->d_jobs = (uint2*)dev_alloc(b->owner, sizeof(uint2) * std::max<size_t>(hj.size(), 1), stream);
    b->d_heads = (uint32_t*)dev_alloc(b->owner, 64, stream);
    const bool wide_lds = slot_words(ma) * 4u <= kSlotLdsBytes;
    if (b->n_wide && !wide_lds)
        b->d_slots = (uint32_t*)dev_alloc(b->owner, size_t(b->grid_wide) * slot_words(ma) * 4u, stream);
    if (!b->d_args || !b->d_jobs || !b->d_heads || (b->n_wide && !wide_lds && !b->d_slots)) {
        batch_free(b);
        set_error("batch: allocation failed");
        return ST_E_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(b->d_args, args.data(), sizeof(TraceArgs) * size_t(n), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !hj.empty())
        e = hipMemcpyAsync(b->d_jobs, hj.data(), sizeof(uint2) * hj.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess && b->n_wide && wide_lds) {
        if (b->deep) e = hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_wide_kernel<32, true>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, int(kSlotLdsBytes));
        else e = hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_wide_kernel<16, true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(kSlotLdsBytes));
    }
    if (e != hipSuccess) { batch_free(b); return device_error(e, "batch: upload"); }
    // one direct frame first: every kernel of the frame is launched (and its
    // code object loaded) outside stream capture, and the frame is checked
    st_status r0 = enqueue_frame(b, stream);
    if (r0 == ST_OK) {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) r0 = device_error(e, "batch: first frame");
    }
    if (r0 != ST_OK) { batch_free(b); return r0; }
    // capture one frame into a graph on a stream of the batch's own
    e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { batch_free(b); return device_error(e, "batch: begin capture"); }
    st_status r = enqueue_frame(b, b->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap_stream, &g);
    if (r != ST_OK) { if (g) (void)hipGraphDestroy(g); batch_free(b); return r; }
    if (e != hipSuccess) { batch_free(b); return device_error(e, "batch: end capture"); }
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { batch_free(b); return device_error(e, "batch: graph instantiate"); }
    *out = b;
    return ST_OK;
}

st_status st_batch_render(st_batch* b, int32_t use_graph, void* stream_v) {
    if (!b) { set_error("batch: NULL"); return ST_E_INVALID; }
    for (size_t i = 0; i < b->scenes.size(); i++)
        if (b->scenes[i]->ab_gen != b->gens[i]) {
            set_error("batch: a scene's A-buffer was rebuilt after the batch was created");
            return ST_E_STALE;
        }
    hipStream_t stream = (hipStream_t)stream_v;
    if (use_graph) {
        hipError_t e = hipGraphLaunch(b->exec, stream);
        return e == hipSuccess ? ST_OK : device_error(e, "batch: graph launch");
    }
    return enqueue_frame(b, stream);
}

st_status st_batch_stats(const st_batch* b, st_stats* out, int32_t cap, void* stream_v) {
    if (!b || !out || cap < int32_t(b->scenes.size())) { set_error("batch stats: bad argument"); return ST_E_INVALID; }
    hipStream_t stream = (hipStream_t)stream_v;
    std::vector<unsigned long long> h(b->scenes.size() * kStatCount);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < b->scenes.size() && e == hipSuccess; i++)
        e = hipMemcpyAsync(h.data() + i * kStatCount, b->scenes[i]->d_stats, kStatCount * 8, hipMemcpyDeviceToHost,
                           stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_error(e, "batch stats");
    for (size_t i = 0; i < b->scenes.size(); i++)
        stats_from_counters(b->scenes[i], h.data() + i * kStatCount, &out[i]);
    return ST_OK;
}

void st_batch_destroy(st_batch* b) {
    if (b) batch_free(b);
}

st_status st_batch_autotune(st_scene* const* scenes, const st_camera* cams, int32_t n, const st_tuning* base,
                            float* const* depths, float* const* normals, int32_t reps, st_tuning* out, float* out_ms,
                            void* stream_v) {
    if (!out || reps < 1) { set_error("batch autotune: NULL out or reps < 1"); return ST_E_INVALID; }
    hipStream_t stream = (hipStream_t)stream_v;
    st_tuning b0;
    if (base) b0 = *base; else st_default_tuning(&b0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) return device_error(he, "batch autotune events");
    const int tiles[3] = {8, 16, 32};
    const int news[4] = {6, 16, 64, 256};
    const float subs[2] = {1.0f / 20.0f, 0.25f};
    float best = INFINITY;
    st_tuning best_t = b0;
    st_status r = ST_OK;
    for (int ti = 0; ti < 3 && r == ST_OK; ti++)
        for (int ni = 0; ni < 4 && r == ST_OK; ni++)
            for (int si = 0; si < 2 && r == ST_OK; si++) {
                st_tuning t = b0;
                t.tile = tiles[ti];
                t.max_new = news[ni];
                t.sub_depth = subs[si];
                st_batch* b = nullptr;
                r = st_batch_create(scenes, cams, n, &t, depths, normals, stream_v, &b);
                if (r != ST_OK) break;
                std::vector<float> ms;
                for (int k = 0; k <= reps && r == ST_OK; k++) {   // first replay warms up
                    he = hipEventRecord(e0, stream);
                    if (he != hipSuccess) { r = device_error(he, "batch autotune record"); break; }
                    r = st_batch_render(b, 1, stream_v);
                    if (r != ST_OK) break;
                    he = hipEventRecord(e1, stream);
                    if (he == hipSuccess) he = hipEventSynchronize(e1);
                    float dt = 0.f;
                    if (he == hipSuccess) he = hipEventElapsedTime(&dt, e0, e1);
                    if (he != hipSuccess) { r = device_error(he, "batch autotune timing"); break; }
                    if (k > 0) ms.push_back(dt);
                }
                st_batch_destroy(b);
                if (r != ST_OK) break;
                std::sort(ms.begin(), ms.end());
                float med = ms[ms.size() / 2];
                if (med < best) { best = med; best_t = t; }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != ST_OK) return r;
    *out = best_t;
    if (out_ms) *out_ms = best;
    return ST_OK;
}

st_status st_trace_batch(st_scene* const* scenes, const st_camera* cams, int32_t n, float* const* depths,
                         float* const* normals, st_stats* stats, void* stream) {
    st_batch* b = nullptr;
    st_status r = st_batch_create(scenes, cams, n, nullptr, depths, normals, stream, &b);
    if (r != ST_OK) return r;
    r = st_batch_render(b, 1, stream);
    if (r == ST_OK && stats) r = st_batch_stats(b, stats, n, stream);
    if (r == ST_OK && !stats) {
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) r = device_error(e, "batch sync");
    }
    st_batch_destroy(b);
    return r;
}

}  // extern "C"
