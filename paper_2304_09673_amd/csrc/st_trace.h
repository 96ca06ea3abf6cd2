// Synchronized tracing of one 8x8 pixel block: the device code shared by the
// single-scene kernels (trace.hip) and the batch kernels (batch.hip).
//
// Synchronized tracing of tile subfrustums (Sections 7, 8 and 9 of Zanni
// 2023; Algorithms 2 and 3), written for CDNA wave64.
//
// One wavefront owns one 8x8 pixel block (64 rays, one per lane) -- the
// paper's 8x8 tile workgroup maps onto a single wave, so the whole
// synchronization of Algorithm 2 is a wave vote and needs no barrier.  The
// wave walks its tile's depth-sorted A-buffer list and cuts the frustum into
// subfrustums [z_begin, z_end] with a fixed active primitive set (Section 8,
// "Tracking active primitives"): exited primitives are dropped, new ones are
// fetched while (no empty gap) and (z_b - z_begin < d) and (at most max_new
// new) and (capacity), and z_end = min(next z_b, max active z_e).  All lanes
// share the set, hence the pruned view, hence every node of every field
// evaluation: node kinds and parameters are wave-uniform (scalar branches,
// scalar loads), only the point differs per lane.
//
// The pruned view is built data-parallel (LCA queries, a wave bitonic sort,
// a merge) plus one short bottom-up pass shared with the host code
// (st_prune.h).  Each ray then sphere-traces its own span [t0, t1] of the
// subfrustum, evaluating the view with the post-order stack machine of
// Algorithm 3.  Steps are clamped at t1 because the pruned field is only
// sign-equivalent to the full field inside the subfrustum.
//
// Stepping: the safe step is f/L with L the proven Lipschitz bound of the
// view.  Once the safe step falls below the probe threshold the ray probes
// forward (probe_len below; never longer than kProbeCapFactor times the
// threshold, so a stretch of negative field at least that long is never
// stepped over); a sign change is bracketed and refined by regula falsi
// (Illinois), and the normal is the normalised forward-mode gradient of the
// view at the root.
//
// Over-relaxed stepping (the variant of Section 10, "Ray processing"; factor
// omega) and the learned step take the step omega f/L and accept it only if
// the unbounding spheres at both ends overlap, f/L + f'/L >= step, which
// certifies the segment under the same Lipschitz bound.  A rejected step
// returns to the plain step from its base; the sphere at the rejected point
// is kept and relaxation stays off until the plain steps reach it, then the
// ray jumps to its far side.  The learned step draws omega per ray from a
// small MLP run on the matrix cores (st_mlp.h); the dump mode runs the plain
// tracer and records, at each step where a relaxed step would be proposed,
// the features and the largest omega of a grid that passes the test.
#pragma once

#include <algorithm>

#include "st_field.h"
#include "st_internal.h"
#include "st_mlp.h"

namespace st {

// ---------------------------------------------------------------------------
// probing near a surface (where the certified step f/L is shorter than the
// probe threshold).  While f falls: three quarters of the secant estimate of
// the distance to the root through the last point (tp, vp) -- where f bends
// down faster than the secant (a concave approach, e.g. where the minimum
// switches to a nearer primitive) the full estimate overshoots the root, and
// a shallow dip behind it can be stepped over whole; while f rises (the ray
// leaves a surface it grazed): twice the last probe.  Growth is at most 4x
// the last probe (hp: the step actually taken, after clamping at the
// subfrustum end), at least eps, at most kProbeCapFactor x the threshold,
// never below the certified step.
constexpr float kProbeCapFactor = 8.0f;

__device__ __forceinline__ float probe_len(float v, float t, float tp, float vp, bool tp_ok, float hp, float eps,
                                           float cap, float safe_s) {
    const bool falling = tp_ok && vp > v;
    const float hb = fmaxf(hp, eps);
    float pr;
    if (falling) pr = fminf(fmaxf(0.75f * v * (t - tp) / (vp - v), eps), 4.f * hb);
    else pr = tp_ok ? 2.f * hb : eps;
    return fmaxf(fminf(pr, cap), safe_s);
}

// ---------------------------------------------------------------------------
// wave helpers
__device__ __forceinline__ int lane_id() { return int(threadIdx.x & 63u); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float unif(float x) { return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x))); }
__device__ __forceinline__ uint32_t rdlane(uint32_t x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ float rdlanef(float x, int l) { return __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(x), l)); }
// lane l of the result is v, every other lane keeps old (v and l uniform)
__device__ __forceinline__ uint32_t wrlane(uint32_t v, int l, uint32_t old) { return int(threadIdx.x & 63u) == l ? v : old; }
__device__ __forceinline__ float wrlanef(float v, int l, float old) { return int(threadIdx.x & 63u) == l ? v : old; }
// orders LDS traffic of the wave (compiler and hardware) between phases
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

// ---------------------------------------------------------------------------
struct TraceArgs {
    const uint32_t* blob;
    const NodePar* par;
    const uint32_t* kill;
    const uint32_t* rmq;
    uint32_t n_nodes;
    const uint32_t* tile_off;
    const uint32_t* tile_cnt;   // per tile: entries kept (the list is [tile_off, tile_off + tile_cnt))
    const uint32_t* e_node;
    const float* e_zin;
    const float* e_zout;
    const uint32_t* tile_ovl;
    const uint4* kslot;        // per node: chain row, 2 x uint4 (killing ancestors, count)
    const uint32_t* tile_order;   // dispatch order of the tiles (fast path)
    const uint32_t* wide;      // [0] count, [1..] tiles
    DevCam cam;
    int ts, tiles_x, tiles_y, sub_x;   // sub_x = ts / 8
    uint32_t ma_fast;
    float eps, probe, probe_cap, d_sub, lip_fixed, omega;   // probe >= eps: safe steps below it probe
    int max_steps, refine_iters, max_new, step_mode;
    float* out_depth;
    float* out_normal;
    uint32_t* out_info;
    unsigned long long* stats;
    unsigned long long* wrec;      // per block (job = tile * sub_x^2 + sub): kWaveStats counters,
                                   // or null: atomics into stats
    const uint32_t* mlp;           // packed step model (learned mode)
    float* dump_x;                 // dump mode: features [cap][8], targets [cap]
    float* dump_t;
    unsigned long long* dump_n;
    unsigned long long dump_cap;
};

// step modes (template parameter of the tracer)
enum { SM_PLAIN = 0, SM_OVER = 1, SM_LEARNED = 2, SM_DUMP = 3, SM_SEGMENT = 4 };

// active-set capacity of the LDS fast path (per wave)
constexpr int kMaFast = 256;
// wide-path slots up to this size are held in LDS (one wave per workgroup)
constexpr size_t kSlotLdsBytes = 80 * 1024;

__host__ __device__ inline uint32_t pow2_at_least(uint32_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}
// 32-bit words of a wide-path slot of capacity ma: active set (node, exit
// depth; two buffers each), vs and view (2 ma each), and the LCA sort array
// (a power of two at least ma)
__host__ __device__ inline size_t slot_words(int ma) { return 8 * size_t(ma) + pow2_at_least(uint32_t(ma)); }

// kernel arguments of one scene (trace.hip)
void fill_trace_args(const st_scene* s, const st_tuning& t, float* depth, float* normal, uint32_t* info,
                     TraceArgs& A);
// wide-path capacity for a scene: a power of two above its largest overlap
int wide_capacity(const st_scene* s);

enum StatIdx {
    S_RAYS = 0, S_HITS, S_UNCONV, S_EVALS, S_GEVALS, S_NODE = 5, S_GNODE = 9, S_STEPS = 13, S_SUBF, S_EMPTY,
    S_VIEWN, S_MAXACT, S_WIDE, S_ACC, S_REJ, S_STALL, S_SMOOTH, S_CYC_MAX, S_CYC_SUM, S_COUNT
};
// words of a block's counter record (S_COUNT rounded up)
constexpr int kWaveStats = 26;
// counters reduced by maximum (the others by sum)
__host__ __device__ constexpr bool stat_is_max(int c) { return c == S_MAXACT || c == S_CYC_MAX; }
static_assert(S_COUNT <= kWaveStats, "counter record too small");

// Per-wave storage of the active set and the view.  Two layouts share the
// tracing code through accessors: LDS arrays of compile-time capacity MA
// (fast path), and a slot of global memory of run-time capacity (tiles whose
// volumes of interest overlap more than the LDS capacity).  Capacities are
// powers of two.  Within one wave, the workgroup-scope fences of wave_sync()
// order both kinds of traffic.
template <int MA>
struct WaveLds {
    uint32_t act_[2][MA];
    float ze_[2][MA];
    uint32_t lca_[MA];
    uint32_t vs_[2 * MA];
    uint32_t view_[2 * MA];
    // buffer b as base + b * MA (an index into the 2-row array would make
    // the compiler keep a table of the two row pointers in scratch memory)
    __device__ __forceinline__ uint32_t* act(int b) { return &act_[0][0] + b * MA; }
    __device__ __forceinline__ float* ze(int b) { return &ze_[0][0] + b * MA; }
    __device__ __forceinline__ uint32_t* lca() { return lca_; }
    __device__ __forceinline__ uint32_t* vs() { return vs_; }
    __device__ __forceinline__ uint32_t* view() { return view_; }
    __device__ __forceinline__ int cap() const { return MA; }
};

// slot_words(ma) 32-bit words per slot (layout in that order)
struct WaveGlob {
    uint32_t* base;
    int ma;
    __device__ __forceinline__ uint32_t* act(int b) { return base + b * ma; }
    __device__ __forceinline__ float* ze(int b) { return reinterpret_cast<float*>(base + (2 + b) * ma); }
    __device__ __forceinline__ uint32_t* vs() { return base + 4 * ma; }
    __device__ __forceinline__ uint32_t* view() { return base + 6 * ma; }
    __device__ __forceinline__ uint32_t* lca() { return base + 8 * ma; }
    __device__ __forceinline__ int cap() const { return ma; }
};

// ---------------------------------------------------------------------------
// field of the pruned view at p (Algorithm 3: post-order stack machine).
// The view entries are wave-uniform.  They are fetched 64 at a time from LDS
// into one VGPR and read with readlane; this is a cross-lane read, so the
// function must be called with every lane of the wave active (inactive rays
// simply evaluate at their stale point and ignore the result).
template <class T, int KS>
__device__ __forceinline__ T eval_view(const uint32_t* view, int len_in, const NodePar* __restrict__ par,
                                       uint32_t n_nodes, const P3<T>& p, uint32_t& sm) {
    T stk[KS];
    T acc = cst(0.f, p.x);
    int sp = 0;
    const int len = int(uni(uint32_t(len_in)));
    for (int base = 0; base < len; base += 64) {
        const uint32_t chunk = view[base + lane_id()];
        const int cnt = int(uni(uint32_t(min(64, len - base))));
        for (int jj = 0; jj < cnt; jj++) {
            uint32_t e = rdlane(chunk, jj);
            uint32_t kind = ventry_kind(e);
            // clamp: a malformed entry reads a wrong node, never outside the array
            const cfloat* q = (const cfloat*)(par[min(ventry_node(e), n_nodes - 1u)].v);
            // Every primitive pushes the running value, the first one the
            // initial value, which is never popped (a view has one operator
            // fewer than primitives).  A view of depth D keeps at most D
            // operands pending above it, at indices 1..D; with KS >= D (KS is
            // at least the tree depth) only index KS wraps, onto that dead
            // slot 0.  An unconditional push is one indexed register move.
            if (kind <= ST_CONE) {
                stk[sp & (KS - 1)] = acc;
                sp++;
                acc = prim_eval<T>(kind, q, p);
            } else {
                sp--;
                acc = op_eval<T>(kind, q, stk[sp & (KS - 1)], acc, sm);
            }
        }
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Segment tracing (Galin et al. 2020, which the paper names as the more robust
// alternative to its empirical Lipschitz constant): the value of the pruned
// view at p and a bound lam on |d f / d tau| over the segment
// p + tau dir, tau in [0, seg] (seg per lane).  Bottom-up: a primitive is a
// signed distance (lam 1); a sharp operator, or a compact one whose two
// operands cannot both reach d_o on the segment (each operand stays within
// its value +- lam seg there), is min / max over the segment (lam = max of
// its operands'); otherwise the compact operator's Lipschitz factor
// 1 + k/(6 d_o - k) multiplies the larger operand bound.  The value is the
// one eval_view returns (same operations).  Called with every lane active.
template <int KS>
__device__ __forceinline__ float eval_view_seg(const uint32_t* view, int len_in, const NodePar* __restrict__ par,
                                               uint32_t n_nodes, const P3<float>& p, float seg, float& lam_out,
                                               uint32_t& sm) {
    float stk[KS], stl[KS];
    float acc = 0.f, lam = 1.f;
    int sp = 0;
    const int len = int(uni(uint32_t(len_in)));
    for (int base = 0; base < len; base += 64) {
        const uint32_t chunk = view[base + lane_id()];
        const int cnt = int(uni(uint32_t(min(64, len - base))));
        for (int jj = 0; jj < cnt; jj++) {
            uint32_t e = rdlane(chunk, jj);
            uint32_t kind = ventry_kind(e);
            const cfloat* q = (const cfloat*)(par[min(ventry_node(e), n_nodes - 1u)].v);
            // push as in eval_view (slot 0 is the dead bottom value)
            if (kind <= ST_CONE) {
                stk[sp & (KS - 1)] = acc;
                stl[sp & (KS - 1)] = lam;
                sp++;
                acc = prim_eval<float>(kind, q, p);
                lam = 1.f;
            } else {
                sp--;
                const float a = stk[sp & (KS - 1)], la = stl[sp & (KS - 1)];
                float m = fmaxf(la, lam);
                if (kind >= ST_SUNION) {
                    const bool blend = a - la * seg <= q[3] && acc - lam * seg <= q[3];
                    if (blend) m *= q[4];
                }
                acc = op_eval<float>(kind, q, a, acc, sm);
                lam = m;
            }
        }
    }
    lam_out = lam;
    return acc;
}

// ---------------------------------------------------------------------------
// device context of the shared bottom-up pass (st_prune.h).  The pass walks
// positions j = 0, 1, ... in order; the data of the current block of 64
// positions sits in four VGPRs (lane l holds position 64c + l) and is read with
// readlane; crossing into the next block reloads it.  The pass stack is held
// across lanes (lane k = stack slot k).  The pass runs with every lane active.
struct DevPruneCtx {
    const uint32_t* vs;
    const uint32_t* gblob;
    const uint32_t* gkill;
    const NodePar* gpar;
    uint32_t n_nodes;
    int m;
    int cur = -1;
    uint32_t cn = 0, cb = 0, ck = 0;
    float cl = 1.f;
    uint32_t s_nu = 0, s_start = 0, s_kill = 0;
    float s_L = 0.f;
    uint32_t* view;
    __device__ void ensure(int j) {
        int c = j >> 6;
        if (c != cur) {
            cur = c;
            int p = c * 64 + lane_id();
            uint32_t v = p < m ? min(vs[p], n_nodes - 1u) : 0u;
            cn = v;
            cb = p < m ? gblob[v] : 0u;
            ck = p < m ? gkill[v] : kNoKill;
            cl = p < m ? gpar[v].v[4] : 1.f;
        }
    }
    __device__ uint32_t node(int j) { ensure(j); return rdlane(cn, j & 63); }
    __device__ uint32_t blob(int j) { ensure(j); return rdlane(cb, j & 63); }
    __device__ uint32_t kill(int j) { ensure(j); return rdlane(ck, j & 63); }
    __device__ float lipf(int j) { ensure(j); return rdlanef(cl, j & 63); }
    __device__ void spush(int sp, uint32_t nu, uint32_t start, float L, uint32_t k) {
        s_nu = wrlane(nu, sp, s_nu);
        s_start = wrlane(start, sp, s_start);
        s_kill = wrlane(k, sp, s_kill);
        s_L = wrlanef(L, sp, s_L);
    }
    __device__ void sget(int sp, uint32_t& nu, uint32_t& start, float& L, uint32_t& k) const {
        nu = rdlane(s_nu, sp);
        start = rdlane(s_start, sp);
        k = rdlane(s_kill, sp);
        L = rdlanef(s_L, sp);
    }
    __device__ void emit(int pos, uint32_t e) {
        if (lane_id() == 0) view[pos] = e;
    }
    __device__ void move(int dst, int src, int len) {
        wave_sync();
        for (int b = 0; b < len; b += 64) {
            int i = b + lane_id();
            uint32_t x = i < len ? view[src + i] : 0u;
            wave_sync();
            if (i < len) view[dst + i] = x;
            wave_sync();
        }
    }
};

// ---------------------------------------------------------------------------
// wave bitonic sort of a[0..np2) (u32) in LDS
__device__ void wave_bitonic(uint32_t* a, int np2) {
    for (int k = 2; k <= np2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            wave_sync();
            for (int i = lane_id(); i < np2; i += 64) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint32_t x = a[i], y = a[ixj];
                    bool up = (i & k) == 0;
                    if ((x > y) == up) { a[i] = y; a[ixj] = x; }
                }
            }
        }
    }
    wave_sync();
}

// number of elements < x in sorted a[0..n)
__device__ __forceinline__ int lower_count(const uint32_t* a, int n, uint32_t x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int m = (lo + hi) >> 1;
        if (a[m] < x) lo = m + 1; else hi = m;
    }
    return lo;
}

// Lowest common ancestors of the consecutive pairs of act[0..n) into
// lca[0..n-1), and into the hash set tab (cleared first).
__device__ void pair_lcas(const TraceArgs& A, const uint32_t* act, int n, uint32_t* lca, uint32_t* tab, int bits) {
    const int lane = lane_id();
    for (int i = lane; i < (1 << bits); i += 64) tab[i] = kNoKill;
    wave_sync();
    for (int i = lane; i < n - 1; i += 64) {
        // a < b always holds for a duplicate-free sorted set; the guard keeps
        // a corrupted set from reading outside the table
        const uint32_t a = act[i], b = act[i + 1];
        const uint32_t l = (a < b && b < A.n_nodes) ? lca_query(A.rmq, A.n_nodes, a, b) : 0u;
        lca[i] = l;
        hinsert(tab, bits, l);
    }
    wave_sync();
}

// Builds the pruned view of the active set S.act(buf)[0..n) into S.view().
//
// First it drops active primitives that cannot reach the root: a primitive
// with a killing ancestor K on its path (an intersection, or a difference
// reached from its right operand) whose other operand holds no active
// primitive is discarded at K, and so is everything below K on that side.
// K has active primitives on both sides exactly when it is the lowest common
// ancestor of two consecutive active primitives (post-order sorted), so the
// test is a lookup of each killing ancestor (chain row: the first
// kKillLevels, then the kill pointers) in the hash set of those LCAs.
// Removing dead primitives leaves the view unchanged; rounds repeat until
// nothing drops, since a drop can leave another killing ancestor one-sided.
// The LCAs of the last round are those of the survivors, which the view
// build needs next.
template <class Mem>
__device__ PruneResult build_view(const TraceArgs& A, Mem& S, int buf, int n) {
    const uint32_t* act = S.act(buf);
    const int lane = lane_id();
    // hash table over vs and view (contiguous, 4 * capacity words, unused
    // until the merge), more than twice the number of LCAs
    uint32_t* tab = S.vs();
    const int bits = 31 - __builtin_clz(uint32_t(4 * S.cap()));
    int m;
    {
        // the two output buffers by a select, not a run-time index into a
        // pointer array (which would live in scratch memory and turn every
        // access through it into a generic-address access)
        uint32_t* const bx0 = S.act(buf ^ 1);
        uint32_t* const bx1 = reinterpret_cast<uint32_t*>(S.ze(buf ^ 1));
        bool lca_ok = false;
        for (int round = 0; round < 8; round++) {
            pair_lcas(A, act, n, S.lca(), tab, bits);
            uint32_t* out = (round & 1) ? bx1 : bx0;
            int kept = 0;
            for (int b = 0; b < n; b += 64) {
                const int s = b + lane;
                const bool in = s < n;
                const uint32_t x = in ? act[s] : 0u;
                const bool keep = in && chain_alive(x, A.kslot, A.kill, A.n_nodes, tab, bits);
                const uint64_t mk = ballot(keep);
                if (keep) out[kept + int(lanes_below(mk))] = x;
                kept += __popcll(mk);
            }
            wave_sync();
            if (kept == n) { lca_ok = true; break; }
            act = out;
            n = kept;
            if (n == 0) break;
        }
        if (n == 0) {
            PruneResult r;
            r.len = 0;
            r.used = 0;
            r.lip = 0.f;
            return r;
        }
        if (!lca_ok) pair_lcas(A, act, n, S.lca(), tab, bits);
    }
    if (n == 1) {
        if (lane == 0) S.vs()[0] = act[0];
        m = 1;
    } else if (n <= 64) {
        // one element per lane: every element's position in post-order by
        // counting (all-pairs compares through readlane; no sort passes)
        const int nl = n - 1;
        const uint32_t a = lane < n ? act[lane] : 0xFFFFFFFFu;
        const uint32_t l = lane < nl ? S.lca()[lane] : 0xFFFFFFFFu;
        uint32_t rl = 0, ca = 0, cl = 0;   // LCAs before l, primitives before l, LCAs before a
        for (int j = 0; j < n; j++) {
            const uint32_t lj = rdlane(l, j), aj = rdlane(a, j);
            if (j < nl) {
                rl += (lj < l || (lj == l && j < lane)) ? 1u : 0u;
                cl += lj < a ? 1u : 0u;
            }
            ca += aj < l ? 1u : 0u;
        }
        wave_sync();
        if (lane < n) S.vs()[lane + int(cl)] = a;
        if (lane < nl) S.vs()[int(rl + ca)] = l;
        m = 2 * n - 1;
    } else {
        // 1. the LCAs of consecutive active primitives (S.lca()), padded to
        //    a power of two
        int nl = n - 1;
        int np2 = 1;
        while (np2 < nl) np2 <<= 1;
        for (int i = nl + lane; i < np2; i += 64) S.lca()[i] = 0xFFFFFFFFu;
        // 2. sort them
        wave_bitonic(S.lca(), np2);
        // 3. merge with the (sorted) primitives into post-order
        for (int i = lane; i < n; i += 64) {
            uint32_t x = act[i];
            S.vs()[i + lower_count(S.lca(), nl, x)] = x;
        }
        for (int i = lane; i < nl; i += 64) {
            uint32_t x = S.lca()[i];
            S.vs()[i + lower_count(act, n, x)] = x;
        }
        m = 2 * n - 1;
    }
    wave_sync();
    // 4. bottom-up pass (usage, killing ancestors, compaction, Lipschitz)
    DevPruneCtx c;
    c.vs = S.vs();
    c.gblob = A.blob;
    c.gkill = A.kill;
    c.gpar = A.par;
    c.n_nodes = A.n_nodes;
    c.m = m;
    c.view = S.view();
    PruneResult r = prune_pass(c, m);
    wave_sync();
    return r;
}

// ---------------------------------------------------------------------------
// Step-model features of a ray at the point t with value v (raw; the model
// normalises them): plain step v/L, contraction v/v_prev, previous step,
// log2(1 + step index), secant slope of f along the ray over L (a cheap
// stand-in for dir . grad f / L), log2(1 + active primitives), t, and
// log2(1 + view length).
__device__ __forceinline__ void step_features(float f[8], float v, float invL, float t, float tp, float vp,
                                              bool tp_ok, int steps, int n_active, int len) {
    const float dt = tp_ok ? fmaxf(t - tp, 1e-12f) : 0.f;
    f[0] = v * invL;
    f[1] = tp_ok && vp > 0.f ? fminf(fmaxf(v / vp, 0.f), 4.f) : 1.f;
    f[2] = dt;
    f[3] = __log2f(1.f + float(steps));
    f[4] = tp_ok ? fminf(fmaxf((v - vp) * invL / dt, -2.f), 2.f) : 0.f;
    f[5] = __log2f(1.f + float(n_active));
    f[6] = t;
    f[7] = __log2f(1.f + float(len));
}

constexpr int kDumpGrid = 12;   // omega = 1.25, 1.5, ..., 4

// Training samples (dump mode): for each lane with `need`, the largest omega
// of the grid whose step (clamped at t1) passes the sphere-overlap test.
// Wave-uniform control flow.
template <int KS>
__device__ void dump_samples(const TraceArgs& A, const uint32_t* view, int len, const Ray& ray, float t, float v,
                             float invL, float t1, bool need, const float f[8]) {
    const float s = v * invL;
    float target = 1.0f;
    for (int j = 1; j <= kDumpGrid; j++) {
        const float om = 1.0f + 0.25f * float(j);
        const float tn = need ? fminf(t + om * s, t1) : t;
        P3<float> p{fmaf(tn, ray.d[0], ray.o[0]), fmaf(tn, ray.d[1], ray.o[1]), fmaf(tn, ray.d[2], ray.o[2])};
        uint32_t sm = 0;
        const float vn = eval_view<float, KS>(view, len, A.par, A.n_nodes, p, sm);
        if (vn > 0.f && (v + vn) * invL >= tn - t) target = om;
    }
    const uint64_t m = ballot(need);
    uint32_t lo = 0u, hi = 0u;
    if (lane_id() == 0) {
        unsigned long long b = atomicAdd(A.dump_n, (unsigned long long)__popcll(m));
        lo = uint32_t(b);
        hi = uint32_t(b >> 32);
    }
    const unsigned long long base = (unsigned long long)rdlane(lo, 0) | ((unsigned long long)rdlane(hi, 0) << 32);
    const unsigned long long idx = base + lanes_below(m);
    if (need && idx < A.dump_cap) {
        for (int k = 0; k < 8; k++) A.dump_x[8 * idx + k] = f[k];
        A.dump_t[idx] = target;
    }
}

// ---------------------------------------------------------------------------
// Counters of one block.  With a record array, lane c stores counter c of
// the block's record (one coalesced write, no atomics: thousands of blocks
// adding into the same few words serialise in the L2 and were the largest
// cost of a frame); the records are summed by a separate kernel when the
// caller asks for statistics.  Without one, lane 0 adds them atomically;
// with neither (a trace without statistics) nothing is written.
__device__ void block_counters(const TraceArgs& A, unsigned long long* cnt, uint32_t job,
                               const unsigned long long (&v)[kWaveStats]) {
    const int lane = lane_id();
    if (A.wrec) {
        unsigned long long mine = 0;
#pragma unroll
        for (int c = 0; c < kWaveStats; c++) mine = lane == c ? v[c] : mine;
        if (lane < kWaveStats) A.wrec[size_t(job) * kWaveStats + size_t(lane)] = mine;
    } else if (cnt != nullptr && lane == 0) {
        for (int c = 0; c < S_COUNT; c++) {
            if (stat_is_max(c)) atomicMax(cnt + c, v[c]);
            else if (v[c]) atomicAdd(cnt + c, v[c]);
        }
    }
}

// Lane modes inside a subfrustum
enum { M_IDLE = 0, M_TRACE = 1, M_REFINE = 2, M_GRAD = 3 };

template <class Mem, int KS, int SM>
__device__ void trace_block(const TraceArgs& A, Mem& S, uint32_t tile, uint32_t sub,
                            unsigned long long* cnt, const uint32_t* tab) {
    constexpr bool kRelax = SM == SM_OVER || SM == SM_LEARNED;
    const int lane = lane_id();
    const int tx = int(tile % uint32_t(A.tiles_x)), ty = int(tile / uint32_t(A.tiles_x));
    const int sx = int(sub % uint32_t(A.sub_x)), sy = int(sub / uint32_t(A.sub_x));
    const int px = tx * A.ts + sx * 8 + (lane & 7);
    const int py = ty * A.ts + sy * 8 + (lane >> 3);
    const bool valid = px < A.cam.w && py < A.cam.h;
    const uint32_t job = tile * uint32_t(A.sub_x * A.sub_x) + sub;
    if (ballot(valid) == 0) {
        const unsigned long long zero[kWaveStats] = {};
        block_counters(A, cnt, job, zero);
        return;
    }
    // the block's duration in shader clock cycles (its counters report the
    // longest and the sum: the launch is set by its slowest blocks)
    const uint64_t clk_start = __builtin_amdgcn_s_memtime();
    Ray ray = pixel_ray(A.cam, px, py);
    const float inv_cos = 1.0f / ray.cosv;

    // per-lane ray state
    float t = 0.f;
    bool done = !valid, hit = false, unconv = false;
    float t_hit = __builtin_inff(), nx = 0.f, ny = 0.f, nz = 0.f;
    int steps = 0;
    uint32_t evals = 0, gevals = 0, smooth = 0;
    float tp = 0.f, vp = 0.f, hp = 0.f;   // last positive point, its value, probe step
    bool tp_ok = false, last_safe = true, refined = false;
    uint32_t n_sub_lane = 0;
    // relaxed steps: base point of the pending step, kept sphere of the last
    // rejected point, relaxation off while t < relax_until
    float tb = 0.f, vb = 0.f, tk = 0.f, vk = -1.f, relax_until = -__builtin_inff();
    bool pend = false;
    uint32_t n_acc = 0, n_rej = 0;

    // wave state (uniform)
    const uint32_t e0 = uni(A.tile_off[tile]), e1 = e0 + uni(A.tile_cnt[tile]);
    uint32_t i = e0;
    int n = 0, buf = 0;
    float z_end = -__builtin_inff();
    uint64_t node_cnt[4] = {0, 0, 0, 0}, gnode_cnt[4] = {0, 0, 0, 0};
    uint32_t n_subf = 0, n_empty = 0, max_act = 0, n_stall = 0;
    uint64_t view_nodes = 0;
    // every turn fetches, drops or closes a subfrustum that the next turn
    // drops from; the bound only guards against a stalled capacity
    uint32_t guard = 4u * (e1 - e0) + 8u;
    // entry depth of list entry i, when known from the last fetch round
    // (saves a dependent global load per turn)
    float zin_i = 0.f;
    bool zin_ok = false;
    // the next fetch window (entries pf_i + lane), loaded at the end of the
    // previous turn's fetch so that its latency overlaps the view build and
    // the stepping
    uint32_t pf_i = 0xFFFFFFFFu, pf_nd = 0u;
    float pf_zb = 0.f, pf_zo = 0.f;

    while (true) {
        if (ballot(!done) == 0) break;
        if (i >= e1 && n == 0) break;
        if (guard-- == 0u) {
            n_stall = 1;
            break;
        }
        // -- drop exited primitives (z_e <= z_end), compact in place; the
        //    remaining ones give the largest exit depth mz.  Elements move only
        //    once something before them has been dropped.
        float mz;
        {
            int kept = 0;
            float mzl = -__builtin_inff();
            for (int b = 0; b < n; b += 64) {
                int s = b + lane;
                bool in = s < n;
                float z = in ? S.ze(buf)[s] : 0.f;
                bool keep = in && z > z_end;
                if (keep) mzl = fmaxf(mzl, z);
                const uint64_t mk = ballot(keep);
                if (mk != ballot(in) || kept != b) {
                    uint32_t a = in ? S.act(buf)[s] : 0u;
                    int dst = kept + int(lanes_below(mk));
                    wave_sync();
                    if (keep) { S.act(buf)[dst] = a; S.ze(buf)[dst] = z; }
                }
                kept += __popcll(mk);
            }
            n = kept;
            mz = wave_max(mzl);
            wave_sync();
        }
        if (i >= e1 && n == 0) break;
        const float z_begin = n > 0 ? z_end : (zin_ok ? zin_i : unif(A.e_zin[i]));
        // -- fetch new primitives, up to 64 per round (lane c considers list
        //    entry i + c), rounds until max_new, a gap, the depth limit or
        //    the capacity stops it
        int fetched = 0;
        while (i < e1 && fetched < A.max_new) {
            uint32_t c = uint32_t(lane);
            bool in = i + c < e1;
            float zb, zo;
            uint32_t nd;
            if (pf_i == i) {
                zb = pf_zb; zo = pf_zo; nd = pf_nd;
            } else {
                zb = in ? A.e_zin[i + c] : __builtin_inff();
                zo = in ? A.e_zout[i + c] : -__builtin_inff();
                nd = in ? A.e_node[i + c] : 0u;
            }
            // exclusive prefix max of exit depths of earlier candidates
            float pm = zo;
            for (int o = 1; o < 64; o <<= 1) {
                float y = __shfl_up(pm, o);
                if (lane >= o) pm = fmaxf(pm, y);
            }
            float pex = __shfl_up(pm, 1);
            if (lane == 0) pex = -__builtin_inff();
            float reach = fmaxf(fmaxf(z_begin, mz), pex);
            bool ok = in && fetched + lane < A.max_new && (n + lane) < S.cap() &&
                      (zb - z_begin < A.d_sub || (lane == 0 && fetched == 0)) && zb <= reach;
            uint64_t okm = ballot(ok);
            const int k = ~okm == 0ull ? 64 : int(__builtin_ctzll(~okm));
            // entry i + k is in this round's window unless all 64 were taken
            zin_ok = k < 64;
            if (k < 64) zin_i = rdlanef(zb, k);   // +inf past the end of the list
            if (k == 0) break;
            // merge the k new primitives (lanes 0..k-1) into the sorted active
            // list: insertion point of each new one in the old list, its rank
            // among the new ones, and for each old element the number of new
            // ones inserted at or before it (histogram of insertion points,
            // then a prefix sum).  Cross-lane reads stay in converged code.
            int nb = buf ^ 1;
            const int ins = lane < k ? lower_count(S.act(buf), n, nd) : n;
            int rk = 0;
            for (int q = 0; q < k; q++) rk += rdlane(nd, q) < nd ? 1 : 0;
            uint32_t* hist = S.lca();   // n + 1 <= capacity words of scratch
            for (int b = lane; b <= n; b += 64) hist[b] = 0u;
            wave_sync();
            if (lane < k) atomicAdd(hist + ins, 1u);
            wave_sync();
            uint32_t carry = 0u;
            for (int b = 0; b < n; b += 64) {
                int s = b + lane;
                bool in_s = s < n;
                uint32_t a = in_s ? S.act(buf)[s] : 0u;
                float az = in_s ? S.ze(buf)[s] : 0.f;
                uint32_t h = in_s ? hist[s] : 0u;
                for (int o = 1; o < 64; o <<= 1) {   // inclusive prefix sum over the chunk
                    uint32_t y = __shfl_up(h, o);
                    if (lane >= o) h += y;
                }
                const uint32_t shift = carry + h;
                carry = rdlane(shift, 63);
                if (in_s) {
                    S.act(nb)[s + int(shift)] = a;
                    S.ze(nb)[s + int(shift)] = az;
                }
            }
            if (lane < k) {
                S.act(nb)[ins + rk] = nd;
                S.ze(nb)[ins + rk] = zo;
            }
            // the new ones also extend the reach
            float nz_ = lane < k ? zo : -__builtin_inff();
            mz = fmaxf(mz, wave_max(nz_));
            buf = nb;
            n += k;
            i += uint32_t(k);
            fetched += k;
            wave_sync();
            if (k < 64) break;
        }
        if (i >= e1) {
            zin_i = __builtin_inff();
            zin_ok = true;
        }
        const float z_next = zin_ok ? zin_i : unif(A.e_zin[i]);
        zin_i = z_next;
        zin_ok = true;
        if (i < e1 && pf_i != i) {
            const uint32_t c = uint32_t(lane);
            const bool in = i + c < e1;
            pf_zb = in ? A.e_zin[i + c] : __builtin_inff();
            pf_zo = in ? A.e_zout[i + c] : -__builtin_inff();
            pf_nd = in ? A.e_node[i + c] : 0u;
            pf_i = i;
        }
        z_end = fminf(z_next, mz);
        max_act = max(max_act, uint32_t(n));
        if (!(z_end > z_begin)) continue;
        n_subf++;

        // -- pruned view of the active set
        PruneResult pr = build_view(A, S, buf, n);
        const float t0 = z_begin * inv_cos, t1 = z_end * inv_cos;
        if (!pr.used) {
            n_empty++;
            if (!done && t < t1) { t = t1; tp_ok = false; }
            continue;
        }
        const int len = int(uni(uint32_t(pr.len)));
        view_nodes += uint64_t(len);
        const float L = A.lip_fixed > 0.f ? A.lip_fixed : pr.lip;
        const float invL = 1.0f / L;
        // kinds in the view (for node counts)
        uint32_t kc[4] = {0, 0, 0, 0};
        for (int j = lane; j < len; j += 64) {
            count_class(kc, ventry_kind(S.view()[j]));
        }
        for (int q = 0; q < 4; q++) kc[q] = uni(wave_sum(kc[q]));

        // -- trace every ray's span of the subfrustum
        int mode = M_IDLE;
        if (!done) {
            if (t < t0) { t = t0; tp_ok = false; }
            if (t < t1) { mode = M_TRACE; n_sub_lane++; }
        }
        pend = false;
        vk = -1.f;
        relax_until = -__builtin_inff();
        float ra = 0.f, fa = 0.f, rb = 0.f, fb = 0.f;   // refinement bracket
        int nref = 0, side = 0;
        uint32_t ev_here = 0;
        uint32_t mlp_it = 0;       // learned step: wave iterations since the last inference
        float om_last = 1.0f;      // learned step: this lane's last proposed factor
        float seg = fmaxf(t1 - t, 0.f);   // segment tracing: candidate segment of the next step
        while (true) {
            bool act = mode == M_TRACE || mode == M_REFINE;
            if (ballot(act) == 0) break;
            P3<float> p{fmaf(t, ray.d[0], ray.o[0]), fmaf(t, ray.d[1], ray.o[1]), fmaf(t, ray.d[2], ray.o[2])};
            uint32_t sm_l = 0;
            float v, lam_seg = L;
            if constexpr (SM == SM_SEGMENT) v = eval_view_seg<KS>(S.view(), len, A.par, A.n_nodes, p, seg, lam_seg, sm_l);
            else v = eval_view<float, KS>(S.view(), len, A.par, A.n_nodes, p, sm_l);
            if (act) {
                ev_here++;
                smooth += sm_l;
            }
            // relaxed-step bookkeeping, in wave-uniform control flow
            bool chk = false, chk_ok = true, need = false;
            float om = A.omega;
            if constexpr (SM != SM_PLAIN && SM != SM_SEGMENT) {
                if constexpr (kRelax) {
                    chk = mode == M_TRACE && pend;
                    chk_ok = !chk || (v > 0.f && (vb + v) * invL >= t - tb);
                }
                const float sp = v * invL;
                need = mode == M_TRACE && chk_ok && v > 0.f && sp >= A.probe && t + sp < t1 && !(t < relax_until);
                if constexpr (SM == SM_LEARNED || SM == SM_DUMP) {
                    if (ballot(need) != 0) {
                        float f[8];
                        step_features(f, v, invL, t, tp, vp, tp_ok, steps, n, len);
                        if constexpr (SM == SM_LEARNED) {
                            // one inference every kMlpEvery iterations of the
                            // wave; in between a ray reuses its last factor
                            if (mlp_it++ % uint32_t(kMlpEvery) == 0u) {
                                om_last = mlp_omega(tab, f);
                                if (!(om_last >= 1.0f)) om_last = 1.0f;   // never below the plain step
                            }
                            om = om_last;
                        }
                        else dump_samples<KS>(A, S.view(), len, ray, t, v, invL, t1, need, f);
                    }
                }
            }
            if (mode == M_TRACE && chk && !chk_ok) {
                // the spheres at both ends do not overlap: plain step from the
                // base; keep the sphere of this point for a later jump
                steps++;
                n_rej++;
                relax_until = t;
                tk = t;
                vk = v;
                pend = false;
                t = tb + vb * invL;
                if (steps >= A.max_steps) {
                    mode = M_IDLE;
                    done = true;
                    unconv = true;
                }
            } else if (mode == M_TRACE && chk && t >= t1) {
                // accepted step that ends on the subfrustum end
                steps++;
                n_acc++;
                pend = false;
                t = t1;
                mode = M_IDLE;
            } else if (mode == M_TRACE) {
                steps++;
                if (chk) {
                    n_acc++;
                    pend = false;
                }
                if (v <= 0.f) {
                    if (!tp_ok || last_safe) {
                        // root at t: the open span before t is root-free
                        t_hit = t;
                        mode = M_GRAD;
                    } else {
                        ra = tp; fa = vp; rb = t; fb = v;
                        nref = 0; side = 0;
                        mode = M_REFINE;
                        refined = true;
                        t = ra + (rb - ra) * (fa / (fa - fb));
                        if (!(t > ra && t < rb)) t = 0.5f * (ra + rb);
                    }
                } else {
                    // certified step: f/L of the view; with segment
                    // tracing also f/lam over the candidate segment, at
                    // most the segment itself (whichever is longer)
                    float safe_s = v * invL;
                    if constexpr (SM == SM_SEGMENT) safe_s = fmaxf(safe_s, fminf(v / lam_seg, seg));
                    float s = safe_s;
                    if (!(safe_s >= A.probe)) {
                        s = probe_len(v, t, tp, vp, tp_ok, hp, A.eps, A.probe_cap, safe_s);
                        hp = fminf(s, t1 - t);   // the step taken (clamped at t1 below)
                    } else {
                        hp = 0.f;
                    }
                    // certified: the step is the safe one (a crossing found
                    // at its end is the root itself)
                    last_safe = !(s > safe_s);
                    tp = t; vp = v; tp_ok = true;
                    float tn = t + s;
                    if constexpr (kRelax) {
                        if (need) {
                            tb = t;
                            vb = v;
                            pend = true;
                            tn = fminf(t + om * s, t1);
                        } else if (vk > 0.f && t < relax_until && t + v * invL >= tk - vk * invL) {
                            // the certified sphere here overlaps the kept one:
                            // the segment up to its far side is root-free
                            const float tj = tk + vk * invL;
                            if (tj > tn) {
                                tn = tj;
                                last_safe = true;
                                hp = 0.f;
                            }
                            vk = -1.f;
                            relax_until = -__builtin_inff();
                        }
                    }
                    if constexpr (SM == SM_SEGMENT) seg = fminf(2.f * s, t1 - tn);   // next candidate
                    if (tn >= t1 && !pend) {
                        t = t1;
                        mode = M_IDLE;
                    } else if (steps >= A.max_steps) {
                        mode = M_IDLE;
                        done = true;
                        unconv = true;
                    } else {
                        t = tn;
                    }
                }
            } else if (mode == M_REFINE) {
                nref++;
                if (v <= 0.f) {
                    rb = t; fb = v;
                    if (side == -1) fa *= 0.5f;   // Illinois
                    side = -1;
                } else {
                    ra = t; fa = v;
                    if (side == 1) fb *= 0.5f;
                    side = 1;
                }
                if (nref >= A.refine_iters || rb - ra <= 1e-6f * fmaxf(1.f, rb)) {
                    t_hit = ra + (rb - ra) * (fa / (fa - fb));
                    if (!(t_hit >= ra && t_hit <= rb)) t_hit = rb;
                    mode = M_GRAD;
                } else {
                    t = ra + (rb - ra) * (fa / (fa - fb));
                    if (!(t > ra && t < rb)) t = 0.5f * (ra + rb);
                }
            }
        }
        // -- normals of the rays that found their root in this subfrustum
        uint32_t g_here = __popcll(ballot(mode == M_GRAD));
        for (int q = 0; q < 4; q++) gnode_cnt[q] += uint64_t(g_here) * kc[q];
        if (g_here != 0) {
            float th = mode == M_GRAD ? t_hit : t;
            P3<Dual> p = make_point(fmaf(th, ray.d[0], ray.o[0]), fmaf(th, ray.d[1], ray.o[1]),
                                    fmaf(th, ray.d[2], ray.o[2]), Dual{});
            uint32_t sm_g = 0;
            Dual g = eval_view<Dual, KS>(S.view(), len, A.par, A.n_nodes, p, sm_g);
            if (mode == M_GRAD) {
                float gn = sqrtf(g.gx * g.gx + g.gy * g.gy + g.gz * g.gz);
                float ig = gn > 0.f ? 1.0f / gn : 0.f;
                nx = g.gx * ig; ny = g.gy * ig; nz = g.gz * ig;
                hit = true;
                done = true;
                gevals++;
            }
        }
        uint32_t tot = uni(wave_sum(ev_here));
        evals += ev_here;
        for (int q = 0; q < 4; q++) node_cnt[q] += uint64_t(tot) * kc[q];
    }

    // outputs
    if (valid) {
        size_t pix = size_t(py) * A.cam.w + px;
        A.out_depth[pix] = hit ? t_hit : __builtin_inff();
        A.out_normal[3 * pix + 0] = hit ? nx : 0.f;
        A.out_normal[3 * pix + 1] = hit ? ny : 0.f;
        A.out_normal[3 * pix + 2] = hit ? nz : 0.f;
        if (A.out_info) {
            uint32_t e = min(evals + gevals, 0xFFFFu);
            A.out_info[pix] = e | (hit ? 1u << 16 : 0u) | (unconv ? 1u << 17 : 0u) | (refined ? 1u << 18 : 0u) |
                              (min(n_sub_lane, 0xFFFu) << 20);
        }
    }
    // counters (one atomic per counter per wave)
    uint32_t rays = __popcll(ballot(valid));
    uint32_t hits = __popcll(ballot(valid && hit));
    uint32_t unc = __popcll(ballot(valid && unconv));
    uint32_t ev = wave_sum(evals + gevals), gev = wave_sum(gevals), st = wave_sum(uint32_t(steps));
    uint32_t smt = wave_sum(smooth);
    uint32_t nacc = 0, nrej = 0;
    if constexpr (kRelax) {
        nacc = wave_sum(n_acc);
        nrej = wave_sum(n_rej);
    }
    unsigned long long v[kWaveStats] = {};
    v[S_RAYS] = rays;
    v[S_HITS] = hits;
    v[S_UNCONV] = unc;
    v[S_EVALS] = ev;
    v[S_GEVALS] = gev;
    v[S_STEPS] = st;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        v[S_NODE + q] = node_cnt[q];
        v[S_GNODE + q] = gnode_cnt[q];
    }
    v[S_SUBF] = n_subf;
    v[S_EMPTY] = n_empty;
    v[S_VIEWN] = view_nodes;
    v[S_MAXACT] = max_act;
    v[S_WIDE] = A.tile_ovl[tile] > A.ma_fast ? 1u : 0u;
    v[S_ACC] = nacc;
    v[S_REJ] = nrej;
    v[S_STALL] = n_stall;
    v[S_SMOOTH] = smt;
    v[S_CYC_MAX] = v[S_CYC_SUM] = __builtin_amdgcn_s_memtime() - clk_start;
    block_counters(A, cnt, job, v);
}


}  // namespace st
