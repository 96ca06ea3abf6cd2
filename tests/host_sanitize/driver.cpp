// Host-only driver of the library's preprocessing code under AddressSanitizer
// and UndefinedBehaviorSanitizer: flatten (validation, post-order relabelling,
// ranges of interest, pruning tables, fast ancestor pointers, bounds), the
// pruned-view pass and the Algorithm 1 traversal, on random valid trees and on
// malformed ones.  Built and run by tests/test_host_sanitize.py; exits non-zero
// on any disagreement, and the sanitizers abort on any memory or UB error.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2304_09673_amd/csrc/st_internal.h"

namespace st {
static std::string g_last;
void set_error(const std::string& msg) { g_last = msg; }
}  // namespace st

namespace {

uint64_t g_rng = 0x9E3779B97F4A7C15ull;
uint32_t rnd() {
    g_rng ^= g_rng << 13;
    g_rng ^= g_rng >> 7;
    g_rng ^= g_rng << 17;
    return uint32_t(g_rng >> 32);
}
float unif(float a, float b) { return a + (b - a) * float(rnd() & 0xFFFFFF) / float(0x1000000); }

st_node primitive() {
    st_node nd{};
    nd.left = nd.right = -1;
    nd.kind = rnd() % 6;
    for (int j = 0; j < 3; j++) nd.p[j] = unif(-1.f, 1.f);
    switch (nd.kind) {
    case ST_SPHERE: nd.p[3] = unif(0.05f, 0.4f); break;
    case ST_BOX:
        for (int j = 3; j < 6; j++) nd.p[j] = unif(0.05f, 0.3f);
        for (int j = 6; j < 10; j++) nd.p[j] = unif(-1.f, 1.f);
        nd.p[6] += 2.f;
        break;
    case ST_CAPSULE:
        for (int j = 3; j < 6; j++) nd.p[j] = nd.p[j - 3] + unif(-0.3f, 0.3f);
        nd.p[6] = unif(0.05f, 0.2f);
        break;
    default:   // torus, cylinder, cone (p[9]: the cone's top radius, 0 allowed)
        nd.p[3] = unif(0.05f, 0.3f);
        nd.p[4] = unif(0.02f, 0.2f);
        for (int j = 5; j < 9; j++) nd.p[j] = unif(-1.f, 1.f);
        nd.p[5] += 2.f;
        if (nd.kind == ST_CONE) nd.p[9] = unif(0.f, 0.3f);
    }
    return nd;
}

// random tree over [lo, hi) leaves appended to nodes; returns its root
int build(std::vector<st_node>& nodes, int n_leaves) {
    if (n_leaves == 1) {
        nodes.push_back(primitive());
        return int(nodes.size()) - 1;
    }
    int nl = 1 + int(rnd() % uint32_t(n_leaves - 1));
    int l = build(nodes, nl), r = build(nodes, n_leaves - nl);
    st_node op{};
    op.kind = ST_UNION + rnd() % 6;
    op.left = l;
    op.right = r;
    op.p[0] = unif(0.02f, 0.2f);
    op.p[1] = (rnd() & 1) ? 0.f : op.p[0] * unif(1.2f, 2.f);
    nodes.push_back(op);
    return int(nodes.size()) - 1;
}

int g_fail = 0;
void check(bool ok, const char* what, int tree) {
    if (!ok) {
        std::fprintf(stderr, "FAIL %s (tree %d)\n", what, tree);
        g_fail++;
    }
}

}  // namespace

int main(int argc, char** argv) {
    const int trees = argc > 1 ? std::atoi(argv[1]) : 300;
    int views = 0;
    for (int t = 0; t < trees; t++) {
        std::vector<st_node> nodes;
        const int leaves = 1 + int(rnd() % 70);
        const int root = build(nodes, leaves);
        // shuffle the caller's node order (children indices follow)
        const int n = int(nodes.size());
        std::vector<int> perm(n);
        for (int i = 0; i < n; i++) perm[i] = i;
        for (int i = n - 1; i > 0; i--) std::swap(perm[i], perm[rnd() % uint32_t(i + 1)]);
        std::vector<st_node> sh(n);
        for (int i = 0; i < n; i++) {
            st_node nd = nodes[i];
            if (nd.left >= 0) { nd.left = perm[nd.left]; nd.right = perm[nd.right]; }
            sh[perm[i]] = nd;
        }
        st_scene s;
        const st_status r = st::flatten_host(sh.data(), n, perm[root], &s);
        check(r == ST_OK, "flatten of a valid tree", t);
        if (r != ST_OK) continue;
        st::subtree_boxes(&s);
        // pruned views of random active sets: the LCA pass and both Algorithm 1 variants agree
        for (int k = 0; k < 12; k++) {
            std::vector<uint32_t> act;
            const uint32_t keep = 1 + rnd() % 8;
            for (uint32_t p : s.h_prims)
                if (rnd() % 8 < keep) act.push_back(p);
            std::vector<uint32_t> v0, v1, v2;
            st::PruneResult pr = st::host_prune(&s, act, v0);
            float l1 = 0.f, l2 = 0.f;
            uint32_t vis1 = 0, vis2 = 0;
            check(st::host_sparse(&s, act, false, v1, l1, vis1) == ST_OK, "parent-pointer traversal", t);
            check(st::host_sparse(&s, act, true, v2, l2, vis2) == ST_OK, "fast-pointer traversal", t);
            std::vector<uint32_t> v0n;
            for (int i = 0; i < pr.len; i++) v0n.push_back(st::ventry_node(v0[size_t(i)]));
            check(v0n == v1 && v1 == v2, "views agree", t);
            check(vis2 <= vis1, "fast pointers visit no more operators", t);
            check(pr.len == 0 || std::fabs(pr.lip - l1) <= 1e-6f * pr.lip, "Lipschitz bounds agree", t);
            views++;
        }
    }
    // malformed input: each must be refused with the right status, never crash
    struct Bad { const char* what; st_status want; };
    for (int t = 0; t < 60; t++) {
        std::vector<st_node> nodes;
        const int root = build(nodes, 2 + int(rnd() % 20));
        const int n = int(nodes.size());
        std::vector<st_node> b = nodes;
        int which = t % 6;
        st_status want = ST_E_TREE;
        int victim = int(rnd() % uint32_t(n));
        switch (which) {
        case 0:   // child out of range
            if (b[root].kind >= ST_UNION) b[root].right = n + 5;
            break;
        case 1:   // cycle: a child points back at the root
            if (b[root].kind >= ST_UNION) b[size_t(b[root].left)] = b[root];
            break;
        case 2:   // NaN parameter
            b[size_t(victim)].p[0] = std::nanf("");
            want = b[size_t(victim)].kind >= ST_UNION && b[size_t(victim)].kind < ST_SUNION ? ST_OK : ST_E_INVALID;
            break;
        case 3:   // unknown kind
            b[size_t(victim)].kind = 9;
            break;
        case 4:   // zero radius / blend radius
            if (b[size_t(victim)].kind == ST_SPHERE) b[size_t(victim)].p[3] = 0.f;
            else if (b[size_t(victim)].kind >= ST_SUNION) b[size_t(victim)].p[0] = 0.f;
            else if (b[size_t(victim)].kind >= ST_TORUS && b[size_t(victim)].kind <= ST_CONE) b[size_t(victim)].p[4] = -1.f;
            else want = ST_OK;
            if (want != ST_OK) want = ST_E_INVALID;
            break;
        default:   // root out of range
            break;
        }
        st_scene s;
        const st_status r = st::flatten_host(b.data(), n, which == 5 ? n : root, &s);
        if (which == 0 || which == 1) {
            check(b[root].kind < ST_UNION ? r == ST_OK || r == ST_E_TREE : r == ST_E_TREE, "malformed tree refused", t);
        } else if (which == 5) {
            check(r != ST_OK, "root out of range refused", t);
        } else {
            check(r == want, "bad parameter status", t);
        }
    }
    std::printf("trees %d, views %d, failures %d\n", trees, views, g_fail);
    return g_fail == 0 ? 0 : 1;
}
