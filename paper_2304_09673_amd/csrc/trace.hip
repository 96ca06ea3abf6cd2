// Single-scene tracing kernels (fast LDS path, wide path) and their launch;
// the per-block tracer is in st_trace.h.
#include <algorithm>
#include <string>

#include "st_trace.h"

namespace st {

// ---------------------------------------------------------------------------
// Fast path: one wave per 8x8 block, 4 waves per workgroup, LDS view of
// capacity MA.  Blocks of tiles that overlap more than MA go to the wide path.
// At least 3 waves per SIMD: the deep-tree and learned-step instances would
// otherwise take more than 170 registers and run 1 or 2 waves per SIMD; the
// few spills this costs are cheaper than the lost latency hiding.
// Waves per workgroup: one (the waves of a workgroup would share nothing,
// and a one-wave workgroup finds room beside other kernels' workgroups, e.g.
// other frames' builds, where a four-wave one with four LDS views waits),
// except for the learned step, whose four waves share the step model's table
// in LDS.
constexpr int fast_waves(int sm) { return sm == SM_LEARNED ? 4 : 1; }

template <int MA, int KS, int SM>
__global__ void __launch_bounds__(64 * fast_waves(SM), 3) trace_fast_kernel(TraceArgs A, uint32_t n_jobs) {
    constexpr int kW = fast_waves(SM);
    __shared__ WaveLds<MA> lds[kW];
    // wave-uniform: the LDS slot address stays scalar
    const int w = kW == 1 ? 0 : int(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    const uint32_t* tab = nullptr;
    if constexpr (SM == SM_LEARNED) {
        __shared__ uint32_t mlp_tab[kMlpTabWords];
        for (int i = int(threadIdx.x); i < kMlpTabWords; i += int(blockDim.x)) mlp_tab[i] = A.mlp[i];
        __syncthreads();
        tab = mlp_tab;
    }
    // Workgroups are dispatched in index order, round-robin over the 8 XCDs:
    // job k is a block of the k-th tile of the longest-first order, so the
    // heaviest tiles start first and spread evenly over the XCDs.
    uint32_t job = blockIdx.x * uint32_t(kW) + uint32_t(w);
    if (job >= n_jobs) return;
    uint32_t spt = uint32_t(A.sub_x * A.sub_x);
    uint32_t tile = A.tile_order[job / spt], sub = job % spt;
    if (A.tile_ovl[tile] > A.ma_fast) return;   // wide path
    trace_block<WaveLds<MA>, KS, SM>(A, lds[w], tile, sub, A.stats, tab);
}

// Wide path: blocks of the listed tiles, one wave per workgroup, each
// workgroup with its own slot of capacity ma: dynamic LDS when it fits
// (InLds), else global memory; the grid strides over the jobs.
template <int KS, int SM, bool InLds>
__global__ void __launch_bounds__(64) trace_wide_kernel(TraceArgs A, uint32_t* slots, int ma) {
    extern __shared__ uint32_t dyn_slot[];
    WaveGlob S{InLds ? dyn_slot : slots + size_t(blockIdx.x) * slot_words(ma), ma};
    // the step-model table is read through the caches here: one wave per
    // workgroup, and LDS is what limits the number of resident waves
    const uint32_t* tab = SM == SM_LEARNED ? A.mlp : nullptr;
    uint32_t n_wide = A.wide[0];
    uint32_t spt = uint32_t(A.sub_x * A.sub_x);
    for (uint32_t job = blockIdx.x; job < n_wide * spt; job += gridDim.x) {
        uint32_t tile = A.wide[1 + job / spt], sub = job % spt;
        trace_block<WaveGlob, KS, SM>(A, S, tile, sub, A.stats, tab);
    }
}

constexpr int kMaDebug = 1024;

// Sums the blocks' counter records into stats[0..S_COUNT) (S_MAXACT: the
// maximum); one workgroup per counter.
__global__ void __launch_bounds__(256) reduce_counters_kernel(const unsigned long long* __restrict__ wrec,
                                                              uint32_t n_jobs, unsigned long long* __restrict__ stats) {
    __shared__ unsigned long long part[256];
    const int c = int(blockIdx.x);
    unsigned long long acc = 0;
    for (uint32_t j = threadIdx.x; j < n_jobs; j += blockDim.x) {
        const unsigned long long x = wrec[size_t(j) * kWaveStats + size_t(c)];
        acc = stat_is_max(c) ? (x > acc ? x : acc) : acc + x;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) {
            const unsigned long long y = part[threadIdx.x + o];
            part[threadIdx.x] = stat_is_max(c) ? (y > part[threadIdx.x] ? y : part[threadIdx.x]) : part[threadIdx.x] + y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) stats[c] = part[0];
}


hipError_t launch_reduce_counters(const unsigned long long* wrec, uint32_t n_jobs, unsigned long long* stats,
                                  hipStream_t stream) {
    hipLaunchKernelGGL(reduce_counters_kernel, dim3(S_COUNT), dim3(256), 0, stream, wrec, n_jobs, stats);
    return hipGetLastError();
}

template <int KS, int SM>
static hipError_t launch_trace(const TraceArgs& A, uint32_t n_jobs, uint32_t wide_grid,
                               uint32_t* slots, int ma, hipStream_t stream) {
    constexpr uint32_t kW = uint32_t(fast_waves(SM));
    hipLaunchKernelGGL((trace_fast_kernel<kMaFast, KS, SM>), dim3((n_jobs + kW - 1) / kW), dim3(64 * kW), 0, stream,
                       A, n_jobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || wide_grid == 0) return e;
    const size_t shm = slot_words(ma) * 4u;
    if (shm <= kSlotLdsBytes) {
        static bool attr_set = false;   // per process; same value every call
        if (!attr_set) {
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&trace_wide_kernel<KS, SM, true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(kSlotLdsBytes));
            if (e != hipSuccess) return e;
            attr_set = true;
        }
        hipLaunchKernelGGL((trace_wide_kernel<KS, SM, true>), dim3(wide_grid), dim3(64), shm, stream, A, slots, ma);
    } else {
        hipLaunchKernelGGL((trace_wide_kernel<KS, SM, false>), dim3(wide_grid), dim3(64), 0, stream, A, slots, ma);
    }
    return hipGetLastError();
}

void fill_trace_args(const st_scene* s, const st_tuning& t, float* depth, float* normal, uint32_t* info,
                     TraceArgs& A) {
    A = TraceArgs{};
    A.blob = s->d_blob;
    A.par = s->d_par;
    A.kill = s->d_kill;
    A.kslot = reinterpret_cast<const uint4*>(s->d_kslot);
    A.rmq = s->d_rmq;
    A.n_nodes = uint32_t(s->n_nodes);
    A.tile_off = s->d_tile_off;
    A.tile_cnt = s->d_tile_cnt;
    A.e_node = s->d_e_node;
    A.e_zin = s->d_e_zin;
    A.e_zout = s->d_e_zout;
    A.tile_ovl = s->d_tile_ovl;
    A.tile_order = s->d_tile_order;
    A.wide = s->d_wide;
    A.cam = s->dcam;
    A.ts = t.tile;
    A.tiles_x = s->tiles_x;
    A.tiles_y = s->tiles_y;
    A.sub_x = t.tile / 8;
    A.ma_fast = uint32_t(s->ab_ma_fast);
    A.eps = t.eps;
    A.probe = std::max(t.probe_step, t.eps);
    A.probe_cap = kProbeCapFactor * A.probe;
    A.d_sub = t.sub_depth * (s->z_max - s->z_min);
    A.lip_fixed = t.lipschitz;
    A.omega = t.omega;
    A.max_steps = t.max_steps;
    A.refine_iters = t.refine_iters;
    A.max_new = std::max(1, std::min(4096, t.max_new));
    A.step_mode = t.step_mode;
    A.out_depth = depth;
    A.out_normal = normal;
    A.out_info = info;
    A.stats = s->d_stats;
}

int wide_capacity(const st_scene* s) {
    // a multiple of 64 above the largest depth overlap, so the active set can
    // always advance
    const uint32_t need = s->max_overlap + 1u;
    return int(std::max<uint32_t>(512u, (need + 63u) / 64u * 64u));
}

st_status trace_device(st_scene* s, const st_tuning& t, float* depth, float* normal, uint32_t* info,
                       hipStream_t stream, const DumpTarget* dump, bool want_stats, const TraceScratch* ext) {
    TraceArgs A;
    fill_trace_args(s, t, depth, normal, info, A);
    int sm = t.step_mode == ST_STEP_OVERRELAX ? SM_OVER
           : t.step_mode == ST_STEP_LEARNED   ? SM_LEARNED
           : t.step_mode == ST_STEP_SEGMENT   ? SM_SEGMENT
                                              : SM_PLAIN;
    if (sm == SM_LEARNED) {
        if (!s->has_model) { set_error("trace: learned step mode without a step model"); return ST_E_INVALID; }
        A.mlp = s->d_mlp;
    }
    if (dump) {
        sm = SM_DUMP;
        A.dump_x = dump->x;
        A.dump_t = dump->t;
        A.dump_n = dump->n;
        A.dump_cap = dump->cap;
    }
    uint32_t spt = uint32_t(A.sub_x * A.sub_x);
    uint32_t n_jobs = uint32_t(s->n_tiles) * spt;
    // one counter record per block, every one written by its block (so a
    // caller's scratch needs no clearing)
    const size_t rec_bytes = size_t(n_jobs) * kWaveStats * 8u;
    if (ext) {
        if (rec_bytes > ext->bytes) {
            set_error("trace: the frame needs " + std::to_string(rec_bytes) + " bytes of counter records, above the " +
                      std::to_string(ext->bytes) + "-byte scratch");
            return ST_E_CAPACITY;
        }
        A.wrec = reinterpret_cast<unsigned long long*>(ext->base);
    } else {
        if (rec_bytes > s->wrec_bytes) {
            dev_free(s, s->d_wrec, stream);
            s->d_wrec = dev_alloc(s, rec_bytes, stream);
            s->wrec_bytes = s->d_wrec ? rec_bytes : 0;
            if (!s->d_wrec) { set_error("trace: counter record allocation failed"); return ST_E_NOMEM; }
        }
        A.wrec = reinterpret_cast<unsigned long long*>(s->d_wrec);
    }
    // evaluation stack: at least the tree depth (views are never deeper)
    const bool shallow = s->depth <= 16;
    uint32_t grid = 0;
    int ma = 512;
    uint32_t* slots = reinterpret_cast<uint32_t*>(s->d_slots);
    if (s->n_wide > 0) {
        ma = wide_capacity(s);
        uint32_t jobs = s->n_wide * spt;
        const bool in_lds = slot_words(ma) * 4u <= kSlotLdsBytes;
        grid = std::min<uint32_t>(jobs, in_lds ? 16384u : 3072u);
        const size_t slot_bytes = slot_words(ma) * 4u;
        if (in_lds) {
            // slots in dynamic LDS
        } else if (ext) {
            // slots after the records; the wide kernel strides over its jobs,
            // so fewer workgroups only take longer
            const size_t off = (rec_bytes + 255u) / 256u * 256u;
            const size_t fit = off < ext->bytes ? (ext->bytes - off) / slot_bytes : 0u;
            if (fit == 0) {
                set_error("trace: no room left in the " + std::to_string(ext->bytes) +
                          "-byte scratch for one wide-path slot of " + std::to_string(slot_bytes) + " bytes");
                return ST_E_CAPACITY;
            }
            grid = uint32_t(std::min<size_t>(grid, fit));
            slots = reinterpret_cast<uint32_t*>(static_cast<char*>(ext->base) + off);
        } else {
            size_t need = size_t(grid) * slot_bytes;
            if (need > s->slots_bytes) {
                dev_free(s, s->d_slots, stream);
                s->d_slots = dev_alloc(s, need, stream);
                s->slots_bytes = s->d_slots ? need : 0;
                if (!s->d_slots) { set_error("trace: wide-path slot allocation failed"); return ST_E_NOMEM; }
            }
            slots = reinterpret_cast<uint32_t*>(s->d_slots);
        }
    }
    // a trace without statistics writes no counters (6 MB of records per
    // 1080p frame otherwise)
    if (!want_stats && !dump) {
        A.wrec = nullptr;
        A.stats = nullptr;
    }
    // every size is checked: launch from here on (the counter reduction
    // overwrites every counter it reports, so the stats words need no clear)
    hipError_t e = hipSuccess;
    switch (sm) {
    case SM_PLAIN:
        e = shallow ? launch_trace<16, SM_PLAIN>(A, n_jobs, grid, slots, ma, stream)
                    : launch_trace<32, SM_PLAIN>(A, n_jobs, grid, slots, ma, stream);
        break;
    case SM_OVER:
        e = shallow ? launch_trace<16, SM_OVER>(A, n_jobs, grid, slots, ma, stream)
                    : launch_trace<32, SM_OVER>(A, n_jobs, grid, slots, ma, stream);
        break;
    case SM_LEARNED:
        e = shallow ? launch_trace<16, SM_LEARNED>(A, n_jobs, grid, slots, ma, stream)
                    : launch_trace<32, SM_LEARNED>(A, n_jobs, grid, slots, ma, stream);
        break;
    case SM_SEGMENT:
        e = shallow ? launch_trace<16, SM_SEGMENT>(A, n_jobs, grid, slots, ma, stream)
                    : launch_trace<32, SM_SEGMENT>(A, n_jobs, grid, slots, ma, stream);
        break;
    default:
        e = launch_trace<32, SM_DUMP>(A, n_jobs, grid, slots, ma, stream);
        break;
    }
    if (e != hipSuccess) return device_error(e, "trace kernels");
    if (want_stats) {
        hipLaunchKernelGGL(reduce_counters_kernel, dim3(S_COUNT), dim3(256), 0, stream, A.wrec, n_jobs, s->d_stats);
        e = hipGetLastError();
        if (e != hipSuccess) return device_error(e, "counter reduction");
    }
    return ST_OK;
}

// ---------------------------------------------------------------------------
// test hook: pruned field of a given active set at points
template <int MA>
__global__ void __launch_bounds__(64) debug_eval_kernel(TraceArgs A, const uint32_t* act_sorted, int n,
                                                         const float* pts, int n_pts, float* out_f, float* out_g,
                                                         int* root_used, uint32_t* view_out) {
    extern __shared__ char dyn[];
    WaveLds<MA>& S = *reinterpret_cast<WaveLds<MA>*>(dyn);
    const int lane = lane_id();
    for (int s = lane; s < n; s += 64) {
        S.act(0)[s] = act_sorted[s];
        S.ze(0)[s] = 0.f;
    }
    wave_sync();
    PruneResult pr = build_view(A, S, 0, n);
    if (lane == 0) {
        root_used[0] = pr.used;
        root_used[1] = pr.len;
        root_used[2] = __float_as_int(pr.lip);
    }
    for (int j = lane; j < pr.len; j += 64) view_out[j] = S.view()[j];
    for (int b = int(blockIdx.x) * 64; b < n_pts; b += int(gridDim.x) * 64) {
        int i = b + lane;
        bool in = i < n_pts;
        float x = in ? pts[3 * i] : 0.f, y = in ? pts[3 * i + 1] : 0.f, z = in ? pts[3 * i + 2] : 0.f;
        if (!pr.used) {
            if (in) {
                out_f[i] = __builtin_inff();
                if (out_g) { out_g[3 * i] = 0.f; out_g[3 * i + 1] = 0.f; out_g[3 * i + 2] = 0.f; }
            }
            continue;
        }
        if (out_g) {
            P3<Dual> p = make_point(x, y, z, Dual{});
            uint32_t sm = 0;
            Dual g = eval_view<Dual, kStack>(S.view(), pr.len, A.par, A.n_nodes, p, sm);
            if (in) { out_f[i] = g.v; out_g[3 * i] = g.gx; out_g[3 * i + 1] = g.gy; out_g[3 * i + 2] = g.gz; }
        } else {
            P3<float> p{x, y, z};
            uint32_t sm = 0;
            float v = eval_view<float, kStack>(S.view(), pr.len, A.par, A.n_nodes, p, sm);
            if (in) out_f[i] = v;
        }
    }
}

st_status debug_eval_device(const st_scene* s, const uint32_t* act_sorted_dev, int n, const float* pts, int n_pts,
                            float* out_f, float* out_g, int* root_used_dev, hipStream_t stream) {
    TraceArgs A{};
    A.blob = s->d_blob;
    A.par = s->d_par;
    A.kill = s->d_kill;
    A.kslot = reinterpret_cast<const uint4*>(s->d_kslot);
    A.rmq = s->d_rmq;
    A.n_nodes = uint32_t(s->n_nodes);
    if (n > kMaDebug) { set_error("debug_eval: active set larger than 1024"); return ST_E_CAPACITY; }
    size_t shm = sizeof(WaveLds<kMaDebug>);
    uint32_t* view_out = reinterpret_cast<uint32_t*>(root_used_dev + 4);
    int grid = std::max(1, std::min(1024, (n_pts + 63) / 64));
    hipLaunchKernelGGL(debug_eval_kernel<kMaDebug>, dim3(grid), dim3(64), shm, stream, A, act_sorted_dev, n, pts,
                       n_pts, out_f, out_g, root_used_dev, view_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ST_OK : device_error(e, "debug_eval_kernel");
}

}  // namespace st
