// Internal (non-ABI) state of a scene and the kernel launchers shared
// between the translation units of the library.
#pragma once

#include <string>
#include <vector>

#include "st_common.h"
#include "st_prune.h"

// axis-aligned boxes of a primitive (support) and of its volume of interest
struct PrimBox {
    double lo[3], hi[3], vlo[3], vhi[3];
};

struct st_scene {
    // tree, post-order numbering
    int32_t n_nodes = 0, n_prims = 0, depth = 0, rmq_levels = 0;
    std::vector<int32_t> post_of_caller;   // caller index -> post-order index
    std::vector<int32_t> caller_of_post;   // post-order index -> caller index
    std::vector<uint32_t> h_blob, h_kill, h_rmq, h_prims;
    std::vector<uint32_t> h_kslot;   // per node: chain row (8 words, see kKillLevels)
    std::vector<st::NodePar> h_par;
    std::vector<float> h_roi;
    std::vector<PrimBox> h_box;   // per primitive, in h_prims order
    // per node, 8 floats: axis-aligned box of the volumes of interest of its
    // subtree (lo xyz, hi xyz, rounded outwards), the first post-order index
    // of its subtree (as bits), 0
    std::vector<float> h_sub;
    // per primitive (h_prims order), 8 words: for each of its first
    // kKillLevels killing ancestors, the child on the other side (kNoKill
    // padding), then 0
    std::vector<uint32_t> h_oside;
    // per node: fast ancestor pointer (kNoNode above the root), and for
    // primitives their index in h_prims (0xFFFFFFFF for operators)
    std::vector<uint32_t> h_fast, h_pslot;
    float extent = 0.f, lipschitz = 1.f;
    float voi_lo[3] = {0, 0, 0}, voi_hi[3] = {0, 0, 0};

    // device copies
    uint32_t* d_blob = nullptr;
    uint32_t* d_kill = nullptr;
    uint32_t* d_kslot = nullptr;     // 8 words per node
    uint32_t* d_rmq = nullptr;
    uint32_t* d_prims = nullptr;     // post-order index of each primitive
    float* d_sub = nullptr;          // h_sub
    uint32_t* d_oside = nullptr;     // h_oside
    uint32_t* d_fast = nullptr;      // h_fast
    uint32_t* d_pslot = nullptr;     // h_pslot
    st::NodePar* d_par = nullptr;
    float* d_roi = nullptr;
    st::Voi* d_voi = nullptr;
    uint64_t device_bytes = 0;

    // A-buffer (per camera)
    bool ab_valid = false;
    st_camera ab_cam{};
    st_tuning ab_tune{};
    st::DevCam dcam{};
    int32_t tiles_x = 0, tiles_y = 0, n_tiles = 0;
    float z_min = 0.f, z_max = 0.f;   // view-depth span of the VOI box
    uint32_t* d_tile_off = nullptr;   // n_tiles + 1
    uint32_t* d_tile_ovl = nullptr;   // per tile max depth overlap
    uint32_t* d_tile_order = nullptr; // tiles by decreasing list length (dispatch order)
    uint32_t* d_tile_cnt = nullptr;   // per tile: entries kept by the tile-level pruning
    uint32_t* d_e_node = nullptr;     // entries, SoA, sorted per tile
    float* d_e_zin = nullptr;
    float* d_e_zout = nullptr;
    uint32_t* d_wide = nullptr;       // list of tiles that need the wide path, [0] = count
    uint32_t* d_misc = nullptr;       // small device counters
    int64_t n_entries = 0, ab_cap = 0;   // entries binned, capacity
    int64_t n_live = 0;                  // entries kept by the tile-level pruning
    uint32_t n_cand = 0;        // (primitive, tile) candidates of the last build
    uint64_t ab_gen = 0;        // bumped by every st_build_abuffer
    uint32_t max_list = 0, max_overlap = 0, n_wide = 0;
    // tiles queued for the long-list pruning, the workgroup sort and the
    // long-list sort in the last sizing build (replays skip empty queues)
    uint32_t n_long_prune = 0, n_sort_queue = 0, n_long_sort = 0;
    int32_t ab_ma_fast = 0, ab_ma_wide = 0;

    // dexel buffer of the ablation tracer: per-pixel CSR offsets, counts and
    // scan scratch (meta), then node, t_in and t_out of every entry (dx)
    void* d_dx_meta = nullptr;
    size_t dx_meta_bytes = 0;
    void* d_dx = nullptr;
    size_t dx_bytes = 0;
    uint32_t n_dexels = 0;

    // wide-path per-workgroup slots (trace)
    void* d_slots = nullptr;
    size_t slots_bytes = 0;
    void* d_wrec = nullptr;           // per-block counter records of the last trace
    size_t wrec_bytes = 0;
    // launch timing of the tile test (st_debug_kernel_timing)
    bool time_test = false;
    std::vector<hipEvent_t> test_events;   // pairs, reused
    size_t test_used = 0;                  // pairs recorded since enabling
    uint64_t cand_pix[3] = {0, 0, 0};      // pixels the per-ray test covers, by kind, last build
    uint32_t n_tested = 0;                 // candidates left for the per-ray test, last build

    // scratch kept between builds
    void* d_scratch = nullptr;
    size_t scratch_bytes = 0;
    void* d_long = nullptr;     // sort scratch of long tile lists
    size_t long_bytes = 0;

    // step model (learned step)
    uint32_t* d_mlp = nullptr;   // packed operand table
    bool has_model = false;

    // device counters for one trace
    unsigned long long* d_stats = nullptr;

    st_allocator alloc{};
    bool has_alloc = false;
};

namespace st {

void set_error(const std::string& msg);
st_status device_error(hipError_t e, const char* where);

void* dev_alloc(st_scene* s, size_t bytes, hipStream_t stream);
void dev_free(st_scene* s, void* p, hipStream_t stream);

// binning.hip
st_status launch_voi(st_scene* s, hipStream_t stream);
st_status build_abuffer_device(st_scene* s, const st_tuning& t, hipStream_t stream, bool replay = false);
hipError_t fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t stream);
// out[0..n) = exclusive prefix sum of in[0..n), *total = the sum (and
// *out_total_slot when non-NULL); scratch holds >= ceil(n/1024)+1 words
void exclusive_scan(const uint32_t* in, uint32_t* out, int n, uint32_t* scratch, uint32_t* total,
                    uint32_t* out_total_slot, hipStream_t stream);

// trace.hip
// training-sample output of the dump mode (device pointers)
struct DumpTarget {
    float* x;                  // [cap][8] features
    float* t;                  // [cap] target omega
    unsigned long long* n;     // samples produced (may exceed cap)
    unsigned long long cap;
};
// caller-provided device scratch for the trace's counter records and
// wide-path slots (instead of the scene's own, allocated on demand)
struct TraceScratch {
    void* base;      // device address, 256-byte aligned
    size_t bytes;
};
// want_stats: sum the blocks' counter records into d_stats after the trace;
// ext: use this scratch and allocate nothing (ST_E_CAPACITY if it is too small)
st_status trace_device(st_scene* s, const st_tuning& t, float* depth, float* normal, uint32_t* info,
                       hipStream_t stream, const DumpTarget* dump = nullptr, bool want_stats = false,
                       const TraceScratch* ext = nullptr);
// sums n_jobs per-block counter records into stats[0..S_COUNT)
hipError_t launch_reduce_counters(const unsigned long long* wrec, uint32_t n_jobs, unsigned long long* stats,
                                  hipStream_t stream);
st_status debug_eval_device(const st_scene* s, const uint32_t* active_post, int n_active,
                            const float* pts, int n_pts, float* out_f, float* out_grad,
                            int* root_used, hipStream_t stream);

// flatten.cpp (host)
st_status flatten_host(const st_node* nodes, int32_t n, int32_t root, st_scene* s);
st_status validate_primitive(const st_node& nd, int i);
// device parameter block and bounds of a primitive with range of interest d
void primitive_params(const st_node& nd, double d, NodePar& par, PrimBox& box);
void subtree_boxes(st_scene* s);
// scene extent and volume-of-interest box from the primitives' boxes
void scene_bounds(st_scene* s);
PruneResult host_prune(const st_scene* s, std::vector<uint32_t> active_post,
                       std::vector<uint32_t>& view);
// Algorithm 1 with parent (fast = false) or fast ancestor pointers, evaluated
// symbolically: the pruned expression in post-order (empty: root unused), its
// Lipschitz bound and the operators visited
st_status host_sparse(const st_scene* s, std::vector<uint32_t> active_post, bool fast, std::vector<uint32_t>& view,
                      float& lip, uint32_t& visited);

constexpr int kStatCount = 48;

// st_stats from the device counters of one trace (api.hip)
void stats_from_counters(const st_scene* s, const unsigned long long* counters, st_stats* out);

}  // namespace st
