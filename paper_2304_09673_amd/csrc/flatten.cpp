// Host preprocessing of a blobtree (the paper's CPU step, run only when the
// tree structure changes; Sections 4, 5 and 7-9):
//  - validation and post-order relabelling (the linearised storage of
//    Section 4 keeps nodes in post-order, so a subtree is a contiguous index
//    range ending at its root);
//  - node bitfields with ignoreMod (Section 9) and parent pointers;
//  - per-node parameter blocks in the device layout;
//  - ranges of interest propagated from the root (Section 5: the root has
//    (-inf, 0]; a compact operator hands its children max(d_o, d_parent), a
//    sharp operator hands them d_parent);
//  - pruning tables: the nearest "killing" ancestor of every node (an
//    intersection, or a difference reached from its right operand: the nodes
//    where the paper cuts fast ancestor pointers) and a sparse table of
//    (depth, parent) over post-order positions for O(1) LCA queries;
//  - the tree's proven Lipschitz bound and bounding boxes.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "st_internal.h"
#include "st_sparse.h"

namespace st {

namespace {

bool finite_params(const st_node& nd, int count) {
    for (int i = 0; i < count; i++)
        if (!std::isfinite(nd.p[i])) return false;
    return true;
}

void quat_axes(const float q_in[4], double axes[3][3]) {
    double w = q_in[0], x = q_in[1], y = q_in[2], z = q_in[3];
    double n = std::sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    // rotation matrix R (row-major); the box axes are its columns
    double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                      {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                      {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) axes[a][c] = R[c][a];
}

}  // namespace

st_status validate_primitive(const st_node& nd, int i) {
    uint32_t k = nd.kind;
    if (nd.left != -1 || nd.right != -1) {
        set_error("primitive " + std::to_string(i) + " has children");
        return ST_E_TREE;
    }
    int cnt = k == ST_SPHERE ? 4 : k == ST_BOX ? 10 : k == ST_CAPSULE ? 7 : k == ST_CONE ? 10 : 9;
    if (!finite_params(nd, cnt)) { set_error("non-finite primitive parameter"); return ST_E_INVALID; }
    if (k == ST_CONE) {
        if (!(nd.p[3] >= 0 && nd.p[9] >= 0 && nd.p[3] + nd.p[9] > 0 && nd.p[4] > 0)) {
            set_error("cone radius < 0, both radii 0 or half height <= 0");
            return ST_E_INVALID;
        }
        double qn = 0;
        for (int j = 5; j < 9; j++) qn += double(nd.p[j]) * nd.p[j];
        if (!(qn > 1e-20)) { set_error("zero quaternion"); return ST_E_INVALID; }
    }
    if (k == ST_TORUS || k == ST_CYLINDER) {
        if (!(nd.p[3] > 0 && nd.p[4] > 0)) {
            set_error(k == ST_TORUS ? "torus radius <= 0" : "cylinder radius or half height <= 0");
            return ST_E_INVALID;
        }
        double qn = 0;
        for (int j = 5; j < 9; j++) qn += double(nd.p[j]) * nd.p[j];
        if (!(qn > 1e-20)) { set_error("zero quaternion"); return ST_E_INVALID; }
    }
    if (k == ST_SPHERE && !(nd.p[3] > 0)) { set_error("sphere radius <= 0"); return ST_E_INVALID; }
    if (k == ST_BOX) {
        if (!(nd.p[3] > 0 && nd.p[4] > 0 && nd.p[5] > 0)) { set_error("box extent <= 0"); return ST_E_INVALID; }
        double qn = 0;
        for (int j = 6; j < 10; j++) qn += double(nd.p[j]) * nd.p[j];
        if (!(qn > 1e-20)) { set_error("zero quaternion"); return ST_E_INVALID; }
    }
    if (k == ST_CAPSULE && !(nd.p[6] > 0)) { set_error("capsule radius <= 0"); return ST_E_INVALID; }
    return ST_OK;
}

void primitive_params(const st_node& nd, double d, NodePar& par, PrimBox& box) {
    float* q = par.v;
    for (int j = 0; j < 16; j++) q[j] = 0.f;
    switch (nd.kind) {
    case ST_SPHERE: {
        for (int j = 0; j < 4; j++) q[j] = nd.p[j];
        for (int j = 0; j < 3; j++) {
            box.lo[j] = double(nd.p[j]) - nd.p[3];
            box.hi[j] = double(nd.p[j]) + nd.p[3];
            box.vlo[j] = box.lo[j] - d;
            box.vhi[j] = box.hi[j] + d;
        }
        break;
    }
    case ST_BOX: {
        double ax[3][3];
        quat_axes(nd.p + 6, ax);
        for (int j = 0; j < 3; j++) q[j] = nd.p[j];
        for (int a = 0; a < 3; a++) {
            for (int c = 0; c < 3; c++) q[4 + 4 * a + c] = float(ax[a][c]);
            q[7 + 4 * a] = nd.p[3 + a];
        }
        for (int j = 0; j < 3; j++) {
            double e = 0, ev = 0;
            for (int a = 0; a < 3; a++) {
                e += std::fabs(ax[a][j]) * nd.p[3 + a];
                ev += std::fabs(ax[a][j]) * (nd.p[3 + a] + d);   // VOI box: offset along the box axes
            }
            box.lo[j] = nd.p[j] - e; box.hi[j] = nd.p[j] + e;
            box.vlo[j] = nd.p[j] - ev; box.vhi[j] = nd.p[j] + ev;
        }
        break;
    }
    case ST_TORUS:
    case ST_CYLINDER:
    case ST_CONE: {
        // local frame of the quaternion; axis 1 is the axis of revolution
        double ax[3][3];
        quat_axes(nd.p + 5, ax);
        for (int j = 0; j < 3; j++) q[j] = nd.p[j];
        for (int a = 0; a < 3; a++)
            for (int c = 0; c < 3; c++) q[4 + 4 * a + c] = float(ax[a][c]);
        q[3] = nd.p[3];
        q[7] = nd.p[4];
        double r_ext = nd.p[3];   // radial extent
        if (nd.kind == ST_TORUS) r_ext = double(nd.p[3]) + nd.p[4];
        if (nd.kind == ST_CONE) {   // top radius, and the inverse length of the side in (rho, y)
            q[11] = nd.p[9];
            const double ex = double(nd.p[9]) - nd.p[3], ey = 2.0 * nd.p[4];
            q[15] = float(1.0 / std::sqrt(ex * ex + ey * ey));
            r_ext = std::max<double>(nd.p[3], nd.p[9]);
        }
        const double ext[3] = {r_ext, double(nd.p[4]), r_ext};
        for (int j = 0; j < 3; j++) {
            double e = 0, ev = 0;
            for (int a = 0; a < 3; a++) {
                e += std::fabs(ax[a][j]) * ext[a];
                ev += std::fabs(ax[a][j]) * (ext[a] + d);   // volume of interest: the local box grown by d
            }
            box.lo[j] = nd.p[j] - e; box.hi[j] = nd.p[j] + e;
            box.vlo[j] = nd.p[j] - ev; box.vhi[j] = nd.p[j] + ev;
        }
        break;
    }
    default: {   // capsule
        double ba[3], bb = 0;
        for (int j = 0; j < 3; j++) { q[j] = nd.p[j]; ba[j] = double(nd.p[3 + j]) - nd.p[j]; q[4 + j] = float(ba[j]); bb += ba[j] * ba[j]; }
        q[3] = nd.p[6];
        q[7] = bb > 0 ? float(1.0 / bb) : 0.f;
        for (int j = 0; j < 3; j++) {
            box.lo[j] = std::min<double>(nd.p[j], nd.p[3 + j]) - nd.p[6];
            box.hi[j] = std::max<double>(nd.p[j], nd.p[3 + j]) + nd.p[6];
            box.vlo[j] = box.lo[j] - d;
            box.vhi[j] = box.hi[j] + d;
        }
    }
    }
}

// Subtree boxes, bottom-up in post-order: a primitive's volume-of-interest
// box, an operator's the union of its children's (right child p - 1, left
// child first(p - 1) - 1).  Doubles are rounded outwards to floats.
void subtree_boxes(st_scene* s) {
    const int n = s->n_nodes;
    s->h_sub.assign(size_t(8) * n, 0.f);
    size_t slot = 0;
    for (int p = 0; p < n; p++) {
        float* b = &s->h_sub[8 * size_t(p)];
        uint32_t first;
        if (blob_prim(s->h_blob[size_t(p)])) {
            const PrimBox& pb = s->h_box[slot++];
            for (int j = 0; j < 3; j++) {
                b[j] = std::nextafter(float(pb.vlo[j]), -INFINITY);
                b[3 + j] = std::nextafter(float(pb.vhi[j]), INFINITY);
            }
            first = uint32_t(p);
        } else {
            const float* r = &s->h_sub[8 * size_t(p - 1)];
            uint32_t fr;
            std::memcpy(&fr, r + 6, 4);
            const float* l = &s->h_sub[8 * size_t(fr - 1)];
            for (int j = 0; j < 3; j++) {
                b[j] = std::min(l[j], r[j]);
                b[3 + j] = std::max(l[3 + j], r[3 + j]);
            }
            std::memcpy(&first, l + 6, 4);
        }
        std::memcpy(b + 6, &first, 4);
    }
    // the other side of each killing ancestor K of a primitive x: K's right
    // child K - 1 when x lies before it (in K's left subtree), else K's left
    // child, which ends just before the right child's subtree
    s->h_oside.assign(size_t(8) * s->h_prims.size(), kNoKill);
    for (size_t i = 0; i < s->h_prims.size(); i++) {
        const uint32_t x = s->h_prims[i];
        for (int k = 0; k < kKillLevels; k++) {
            const uint32_t K = s->h_kslot[8 * size_t(x) + size_t(k)];
            if (K == kNoKill) break;
            const uint32_t rc = K - 1u;
            uint32_t first_r;
            std::memcpy(&first_r, &s->h_sub[8 * size_t(rc) + 6], 4);
            s->h_oside[8 * i + size_t(k)] = x < first_r ? rc : first_r - 1u;
        }
        s->h_oside[8 * i + 7] = 0u;
    }
}

void scene_bounds(st_scene* s) {
    double ext_lo[3] = {INFINITY, INFINITY, INFINITY}, ext_hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double voi_lo[3] = {INFINITY, INFINITY, INFINITY}, voi_hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (const PrimBox& b : s->h_box)
        for (int j = 0; j < 3; j++) {
            ext_lo[j] = std::min(ext_lo[j], b.lo[j]); ext_hi[j] = std::max(ext_hi[j], b.hi[j]);
            voi_lo[j] = std::min(voi_lo[j], b.vlo[j]); voi_hi[j] = std::max(voi_hi[j], b.vhi[j]);
        }
    double e = 0;
    for (int j = 0; j < 3; j++) {
        e = std::max(e, ext_hi[j] - ext_lo[j]);
        s->voi_lo[j] = float(voi_lo[j]);
        s->voi_hi[j] = float(voi_hi[j]);
    }
    s->extent = float(e);
}

st_status flatten_host(const st_node* nodes, int32_t n, int32_t root, st_scene* s) {
    if (!nodes || n <= 0 || root < 0 || root >= n) {
        set_error("flatten: NULL nodes, n <= 0 or root out of range");
        return ST_E_INVALID;
    }
    if (uint32_t(n) >= kMaxNodes) {
        set_error("flatten: too many nodes");
        return ST_E_CAPACITY;
    }
    // validate kinds and parameters
    for (int i = 0; i < n; i++) {
        const st_node& nd = nodes[i];
        uint32_t k = nd.kind;
        if (is_prim_kind(k)) {
            st_status r = validate_primitive(nd, i);
            if (r != ST_OK) return r;
        } else if (is_op_kind(k)) {
            if (nd.left < 0 || nd.left >= n || nd.right < 0 || nd.right >= n || nd.left == nd.right) {
                set_error("flatten: operator " + std::to_string(i) + " has invalid children");
                return ST_E_TREE;
            }
            if (is_compact_kind(k)) {
                if (!finite_params(nd, 2)) { set_error("flatten: non-finite blend parameter"); return ST_E_INVALID; }
                double kk = nd.p[0], d = nd.p[1] > 0 ? nd.p[1] : 7.0 * kk / 6.0;
                if (!(kk > 0)) { set_error("flatten: blend radius k <= 0"); return ST_E_INVALID; }
                if (!(6.0 * d - kk > 0)) { set_error("flatten: 6 d_o - k <= 0"); return ST_E_INVALID; }
            }
        } else {
            set_error("flatten: unknown node kind " + std::to_string(k));
            return ST_E_TREE;
        }
    }

    // post-order walk from the root; every node must be reached exactly once
    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<int32_t> parent(n, -1), depth(n, 0);
    std::vector<char> seen(n, 0);
    std::vector<std::pair<int32_t, int>> stk;
    stk.reserve(64);
    stk.push_back({root, 0});
    seen[root] = 1;
    int maxd = 0;
    while (!stk.empty()) {
        auto& top = stk.back();
        int32_t v = top.first;
        const st_node& nd = nodes[v];
        if (is_prim_kind(nd.kind) || top.second == 2) {
            order.push_back(v);
            stk.pop_back();
            continue;
        }
        int32_t c = top.second == 0 ? nd.left : nd.right;
        top.second++;
        if (seen[c]) { set_error("flatten: node reached twice (cycle or shared child)"); return ST_E_TREE; }
        seen[c] = 1;
        parent[c] = v;
        depth[c] = depth[v] + 1;
        maxd = std::max(maxd, depth[c]);
        if (maxd > kMaxDepth) { set_error("flatten: tree deeper than 31 levels"); return ST_E_TREE; }
        stk.push_back({c, 0});
    }
    if (int32_t(order.size()) != n) { set_error("flatten: not every node is reachable from the root"); return ST_E_TREE; }

    s->n_nodes = n;
    s->depth = maxd;
    s->post_of_caller.assign(n, -1);
    s->caller_of_post.assign(n, -1);
    for (int p = 0; p < n; p++) {
        s->caller_of_post[p] = order[p];
        s->post_of_caller[order[p]] = p;
    }
    s->h_blob.assign(n, 0);
    s->h_kill.assign(n, kNoKill);
    s->h_par.assign(n, NodePar{});
    s->h_roi.assign(n, 0.f);
    s->h_prims.clear();

    std::vector<double> roi(n, 0.0), lip(n, 1.0);
    // top-down: roi, Lipschitz products, kill pointers (parents come later in post-order)
    for (int p = n - 1; p >= 0; p--) {
        int32_t c = order[p];
        const st_node& nd = nodes[c];
        int32_t pc = parent[c];
        uint32_t pp = pc >= 0 ? uint32_t(s->post_of_caller[pc]) : kNoNode;
        bool is_left = pc >= 0 && nodes[pc].left == c;
        s->h_blob[p] = blob_pack(is_prim_kind(nd.kind), nd.kind, is_op_kind(nd.kind) ? ignore_of(nd.kind) : 0u,
                                 is_left, pp);
        if (pc < 0) {
            roi[p] = 0.0;
            lip[p] = 1.0;
            s->h_kill[p] = kNoKill;
        } else {
            const st_node& pn = nodes[pc];
            double dp = roi[pp], lf = 1.0;
            if (is_compact_kind(pn.kind)) {
                double kk = pn.p[0], d = pn.p[1] > 0 ? pn.p[1] : 7.0 * kk / 6.0;
                dp = std::max(dp, d);
                lf = 1.0 + kk / (6.0 * d - kk);
            }
            roi[p] = dp;
            lip[p] = lip[pp] * lf;
            uint32_t im = ignore_of(pn.kind);
            bool kills = is_left ? (im & 1u) != 0 : (im & 2u) != 0;
            s->h_kill[p] = kills ? pp : s->h_kill[pp];
        }
        s->h_roi[p] = float(roi[p]);
    }
    // fast ancestor pointers (Algorithm 1's long jumps; the ablation tracer)
    s->h_fast.assign(n, kNoNode);
    for (int p = 0; p < n; p++) s->h_fast[p] = fast_ancestor(s->h_blob.data(), uint32_t(p));
    // chain rows: a node's first kKillLevels killing ancestors, nearest first
    // (following the kill pointers from node to node visits every killing
    // ancestor on the path to the root), padded with kNoKill, then their count
    s->h_kslot.assign(size_t(8) * n, kNoKill);
    for (int p = 0; p < n; p++) {
        uint32_t* row = &s->h_kslot[8 * size_t(p)];
        uint32_t v = uint32_t(p), lev = 0;
        while (lev < uint32_t(kKillLevels) && s->h_kill[v] < uint32_t(n)) {
            v = s->h_kill[v];
            row[lev++] = v;
        }
        row[7] = lev;
    }

    // parameters, bounds
    double Lmax = 1.0;
    int nprim = 0;
    s->h_box.clear();
    for (int p = 0; p < n; p++) {
        const st_node& nd = nodes[order[p]];
        float* q = s->h_par[p].v;
        if (is_prim_kind(nd.kind)) {
            PrimBox box;
            primitive_params(nd, roi[p], s->h_par[p], box);
            s->h_box.push_back(box);
            s->h_prims.push_back(uint32_t(p));
            nprim++;
            Lmax = std::max(Lmax, lip[p]);
        } else if (is_compact_kind(nd.kind)) {
            double kk = nd.p[0], dd = nd.p[1] > 0 ? nd.p[1] : 7.0 * kk / 6.0;
            q[0] = float(kk);
            q[1] = float(1.0 / kk);
            q[2] = float(6.0 * kk / (6.0 * dd - kk));
            q[3] = float(dd);
            q[4] = float(1.0 + kk / (6.0 * dd - kk));
            q[5] = float(kk / 6.0);
        } else {
            q[4] = 1.f;
        }
    }
    s->n_prims = nprim;
    s->h_pslot.assign(n, 0xFFFFFFFFu);
    for (int i = 0; i < nprim; i++) s->h_pslot[s->h_prims[size_t(i)]] = uint32_t(i);
    s->lipschitz = float(Lmax);
    scene_bounds(s);
    subtree_boxes(s);

    // sparse table over post-order positions of (depth << 24 | parent)
    int levels = 1;
    while ((1 << levels) <= n) levels++;
    s->rmq_levels = levels;
    s->h_rmq.assign(size_t(levels) * n, 0xFFFFFFFFu);
    for (int p = 0; p < n; p++) {
        int32_t c = order[p];
        int32_t pc = parent[c];
        s->h_rmq[p] = pc < 0 ? 0xFFFFFFFFu
                             : (uint32_t(depth[c]) << 24) | uint32_t(s->post_of_caller[pc]);
    }
    for (int k = 1; k < levels; k++) {
        int half = 1 << (k - 1);
        for (int x = 0; x + (1 << k) <= n; x++) {
            uint32_t a = s->h_rmq[size_t(k - 1) * n + x], b = s->h_rmq[size_t(k - 1) * n + x + half];
            s->h_rmq[size_t(k) * n + x] = std::min(a, b);
        }
    }
    return ST_OK;
}

namespace {

struct HostCtx {
    const st_scene* s;
    const std::vector<uint32_t>* vs;
    std::vector<uint32_t>* out;
    uint32_t st_nu[kStack + 2], st_start[kStack + 2], st_kill[kStack + 2];
    float st_L[kStack + 2];
    uint32_t node(int j) const { return (*vs)[j]; }
    uint32_t blob(int j) const { return s->h_blob[(*vs)[j]]; }
    uint32_t kill(int j) const { return s->h_kill[(*vs)[j]]; }
    float lipf(int j) const { return s->h_par[(*vs)[j]].v[4]; }
    void spush(int sp, uint32_t nu, uint32_t start, float L, uint32_t k) {
        st_nu[sp] = nu; st_start[sp] = start; st_L[sp] = L; st_kill[sp] = k;
    }
    void sget(int sp, uint32_t& nu, uint32_t& start, float& L, uint32_t& k) const {
        nu = st_nu[sp]; start = st_start[sp]; L = st_L[sp]; k = st_kill[sp];
    }
    void emit(int pos, uint32_t e) { (*out)[pos] = e; }
    void move(int dst, int src, int len) {
        for (int i = 0; i < len; i++) (*out)[dst + i] = (*out)[src + i];
    }
};

}  // namespace

// Host version of the tracer's view build: same LCA query, same merge, same
// bottom-up pass.  active_post: post-order indices of active primitives.
PruneResult host_prune(const st_scene* s, std::vector<uint32_t> act, std::vector<uint32_t>& view) {
    PruneResult r{0, 0, 0.f};
    view.clear();
    if (act.empty()) return r;
    std::sort(act.begin(), act.end());
    std::vector<uint32_t> lcas;
    for (size_t i = 0; i + 1 < act.size(); i++)
        lcas.push_back(lca_query(s->h_rmq.data(), uint32_t(s->n_nodes), act[i], act[i + 1]));
    std::sort(lcas.begin(), lcas.end());
    std::vector<uint32_t> vs;
    std::merge(act.begin(), act.end(), lcas.begin(), lcas.end(), std::back_inserter(vs));
    view.assign(vs.size(), 0u);
    HostCtx c;
    c.s = s;
    c.vs = &vs;
    c.out = &view;
    r = prune_pass(c, int(vs.size()));
    view.resize(size_t(r.len));
    return r;
}

namespace {

// Symbolic evaluation of the sparse traversal: a value is a pruned
// expression (post-order node list and its Lipschitz bound) or "unused".
struct SymEval {
    typedef int V;   // index into pool, -1: unused
    const st_scene* s;
    std::vector<std::vector<uint32_t>> pool;
    std::vector<float> lip;
    int make(std::vector<uint32_t> e, float L) {
        pool.push_back(std::move(e));
        lip.push_back(L);
        return int(pool.size()) - 1;
    }
    V none() { return -1; }
    V prim(uint32_t node) { return make({node}, 1.f); }
    V single(uint32_t op, V v, bool from_left) {
        if (v < 0) return -1;
        return single_passes(s->h_blob[op], from_left) ? v : -1;
    }
    V op(uint32_t op, V a, V b) {
        if (a < 0) return single(op, b, false);
        if (b < 0) return single(op, a, true);
        std::vector<uint32_t> e = pool[size_t(a)];
        e.insert(e.end(), pool[size_t(b)].begin(), pool[size_t(b)].end());
        e.push_back(op);
        return make(std::move(e), s->h_par[op].v[4] * std::max(lip[size_t(a)], lip[size_t(b)]));
    }
};

struct HostTree {
    const st_scene* s;
    bool fast;
    uint32_t blob(uint32_t n) const { return s->h_blob[n]; }
    uint32_t anc(uint32_t n) const { return fast ? s->h_fast[n] : blob_anc(s->h_blob[n]); }
};

struct HostAct {
    const std::vector<uint32_t>* a;
    size_t i = 0;
    bool next(uint32_t& n) {
        if (i >= a->size()) return false;
        n = (*a)[i++];
        return true;
    }
};

}  // namespace

st_status host_sparse(const st_scene* s, std::vector<uint32_t> act, bool fast, std::vector<uint32_t>& view,
                      float& lip, uint32_t& visited) {
    std::sort(act.begin(), act.end());
    SymEval ev;
    ev.s = s;
    HostTree tr{s, fast};
    HostAct ac;
    ac.a = &act;
    bool overflow = false;
    visited = 0;
    int r = fast ? sparse_traverse<true, kStack>(tr, ac, ev, visited, overflow)
                 : sparse_traverse<false, kStack>(tr, ac, ev, visited, overflow);
    if (overflow) { set_error("sparse traversal: stack overflow or unfinished traversal"); return ST_E_CAPACITY; }
    view.clear();
    lip = 0.f;
    if (r >= 0) {
        view = ev.pool[size_t(r)];
        lip = ev.lip[size_t(r)];
    }
    return ST_OK;
}

}  // namespace st
