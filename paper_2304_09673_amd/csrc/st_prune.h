// Pruned tree view of an active primitive set (Sections 7-9 of Zanni 2023).
//
// The paper builds the view with a sparse bottom-up traversal driven by
// ancestor pointers, run by one thread per workgroup (Algorithm 1, fast
// ancestor pointers cut at intersections and at differences reached from the
// right, plus the usage stack of Section 9).  Here the same view is obtained
// in two data-parallel steps and one short sequential pass:
//
//  1. The nodes with two active operands are exactly the lowest common
//     ancestors of consecutive active primitives (primitives sorted by
//     post-order index).  Each LCA is an O(1) range-minimum query over the
//     post-order depth array (sparse table of (depth << 24 | parent)).
//  2. Primitives and LCAs, merged in post-order, form the "virtual tree"; its
//     post-order is the post-order of the full tree restricted to them.
//  3. One bottom-up pass (this file, shared by host and device) applies the
//     ignoreMod rules: an operand is unused if its own usage is 0 or if a node
//     strictly between it and its virtual parent discards a lone operand
//     (an intersection, or a difference reached from the right).  The
//     nearest such "killing" ancestor of every node is precomputed at
//     flatten time, so the test is one comparison of post-order indices.
//     The operator's op_type is ((~b & ignoreMod) == 0) ? b : 0 with
//     b = (leftUsed << 1) | rightUsed; the paper's reserved op types
//     (0: +inf, 1: right, 2: left) are applied by deleting the dropped
//     subtree from the output, so the evaluated view holds only primitives
//     and operators with both operands used.
//
// The view's Lipschitz bound is the maximum over root-to-leaf paths of the
// product of the operators' factors (1 + k/(6 d_o - k) for compact operators,
// 1 for sharp ones).
#pragma once

#include "st_common.h"

namespace st {

// Lowest common ancestor of nodes a < b (post-order indices) that are not
// ancestors of one another.  The node of least depth in the post-order range
// [a, b-1] is the left child of the LCA and is the only node of that depth in
// the range, so the packed minimum carries the LCA in its low 24 bits.
HD uint32_t lca_query(const uint32_t* rmq, uint32_t n_nodes, uint32_t a, uint32_t b) {
    uint32_t len = b - a;
    uint32_t k = 31u - __builtin_clz(len);
    uint32_t x = rmq[size_t(k) * n_nodes + a];
    uint32_t y = rmq[size_t(k) * n_nodes + (b - (1u << k))];
    return (x < y ? x : y) & 0xFFFFFFu;
}

// Hash set of node indices in LDS or global memory: open addressing, linear
// probing, kNoKill marks an empty slot.  The table has 2^bits slots and is
// filled to less than half, so every probe sequence reaches an empty slot.
__device__ __forceinline__ uint32_t hslot(uint32_t k, int bits) { return (k * 2654435761u) >> (32 - bits); }

__device__ __forceinline__ void hinsert(uint32_t* tab, int bits, uint32_t k) {
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t h = hslot(k, bits);
    while (true) {
        const uint32_t old = atomicCAS(tab + h, kNoKill, k);
        if (old == kNoKill || old == k) return;
        h = (h + 1u) & mask;
    }
}

// membership of k, given the content t of its home slot (read in advance)
__device__ __forceinline__ bool hfind(const uint32_t* tab, int bits, uint32_t k, uint32_t t) {
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t h = hslot(k, bits);
    while (t != k && t != kNoKill) {
        h = (h + 1u) & mask;
        t = tab[h];
    }
    return t == k;
}

// Whether primitive x survives every killing ancestor on its path, given the
// hash set of the nodes with active primitives on both sides (the LCAs of
// consecutive active primitives): its chain row lists the first kKillLevels
// killing ancestors (kNoKill padding), the kill pointers continue a longer
// chain (ancestors are later in post-order, so the walk ends).  The home
// slots of the row's ancestors are read together.
__device__ __forceinline__ bool chain_alive(uint32_t x, const uint4* __restrict__ kslot,
                                            const uint32_t* __restrict__ kill, uint32_t n_nodes,
                                            const uint32_t* tab, int bits) {
    const uint4* row = kslot + size_t(min(x, n_nodes - 1u)) * 2u;
    const uint4 r0 = row[0], r1 = row[1];
    const uint32_t K[kKillLevels] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z};
    uint32_t t[kKillLevels];
#pragma unroll
    for (int j = 0; j < kKillLevels; j++) t[j] = K[j] != kNoKill ? tab[hslot(K[j], bits)] : kNoKill;
    bool keep = true;
#pragma unroll
    for (int j = 0; j < kKillLevels; j++)
        if (K[j] != kNoKill) keep = keep && hfind(tab, bits, K[j], t[j]);
    uint32_t v = keep && r1.w == uint32_t(kKillLevels) ? K[kKillLevels - 1] : kNoKill;
    while (v < n_nodes) {
        const uint32_t u = kill[v];
        if (!(u < n_nodes && u > v)) break;
        if (!hfind(tab, bits, u, tab[hslot(u, bits)])) { keep = false; break; }
        v = u;
    }
    return keep;
}

struct PruneResult {
    int len;     // number of view entries (0 when the root is unused)
    int used;    // 1 when the pruned root is used
    float lip;   // Lipschitz bound of the view
};

// Bottom-up pass over the m nodes of the virtual tree in post-order.
// Ctx supplies the per-position data and the storage:
//   uint32_t node(j), blob(j), kill(j); float lipf(j);
//   void spush(sp, uint32_t node_used, uint32_t start, float L, uint32_t kill);
//   void sget(sp, uint32_t& node_used, uint32_t& start, float& L, uint32_t& kill);
//   void emit(pos, uint32_t entry); void move(dst, src, len)
// Stack entries: node index | used << 31, first output position of the
// node's subtree, Lipschitz bound of the subtree, the node's nearest killing
// ancestor.
template <class Ctx>
__host__ __device__ inline PruneResult prune_pass(Ctx& c, int m) {
    int sp = 0;
    int cur = 0;
    for (int j = 0; j < m; j++) {
        uint32_t v = c.node(j);
        uint32_t b = c.blob(j);
        if (blob_prim(b)) {
            c.emit(cur, ventry(v, blob_op(b)));
            c.spush(sp, v | 0x80000000u, uint32_t(cur), 1.0f, c.kill(j));
            sp++;
            cur++;
            continue;
        }
        uint32_t rn, rs, ln, ls, rk, lk;
        float rL, lL;
        c.sget(sp - 1, rn, rs, rL, rk);
        c.sget(sp - 2, ln, ls, lL, lk);
        sp -= 2;
        // a killing ancestor strictly below v discards the lone operand
        uint32_t lu = ((ln >> 31) != 0 && !(lk < v)) ? 1u : 0u;
        uint32_t ru = ((rn >> 31) != 0 && !(rk < v)) ? 1u : 0u;
        uint32_t bits = (lu << 1) | ru;
        uint32_t im = blob_ignore(b);
        uint32_t op_type = ((~bits & im) == 0u) ? bits : 0u;
        uint32_t kv = c.kill(j);
        if (op_type == 3u) {
            float L = (lL > rL ? lL : rL) * c.lipf(j);
            c.emit(cur, ventry(v, blob_op(b)));
            cur++;
            c.spush(sp, v | 0x80000000u, ls, L, kv);
        } else if (op_type == 2u) {          // left operand only: drop the right subtree
            cur = int(rs);
            c.spush(sp, v | 0x80000000u, ls, lL, kv);
        } else if (op_type == 1u) {          // right operand only: drop the left subtree
            int len = cur - int(rs);
            c.move(int(ls), int(rs), len);
            cur = int(ls) + len;
            c.spush(sp, v | 0x80000000u, ls, rL, kv);
        } else {                             // unused: +inf, nothing to evaluate
            cur = int(ls);
            c.spush(sp, v, ls, 0.0f, kv);
        }
        sp++;
    }
    PruneResult r;
    uint32_t tn, ts, tk;
    float tL;
    c.sget(sp - 1, tn, ts, tL, tk);
    r.used = ((tn >> 31) != 0 && tk == kNoKill) ? 1 : 0;
    r.len = r.used ? cur : 0;
    r.lip = r.used ? tL : 0.0f;
    return r;
}

}  // namespace st
