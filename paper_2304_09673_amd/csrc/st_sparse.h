// Sparse bottom-up blobtree traversal with direct evaluation (Algorithm 1 of
// Zanni 2023, Section 7): starting from each active primitive in increasing
// post-order address, the traversal climbs ancestor pointers, evaluating each
// visited operator, until the next ancestor lies after the next unprocessed
// active primitive (the shadowing condition), where it stacks the partial
// result.  An operator whose two operands are active pops the stacked left
// operand; an operator reached by one operand alone applies its ignoreMod
// rule (Section 9): a union passes the operand through, an intersection, or a
// difference reached from its right operand, returns "unused" (+inf), a
// difference reached from its left passes it through.
//
// Two ancestor pointers (the ablation of the paper's Table 1):
//  * parent pointers: every ancestor of an active primitive is visited;
//  * fast ancestor pointers: a node points past the ancestors it reaches from
//    the same side (left or right) as itself, stopping at an intersection, a
//    difference reached from the right, or the first ancestor that lies on the
//    other side of its own parent.  The printed recursion stops at the parent
//    when the sides agree, which drops operators; the stopping rule here is the
//    reading that keeps every operator (checked exhaustively on small trees by
//    the host tests).  Before every climb the pointer is clamped to the
//    ancestor stored with the stacked operand, and a stacked operand is also
//    popped at a left-child operator whose own fast pointer reaches at least as
//    far as the stacked one (the paper's second pop condition).
//
// The traversal is generic: Tree gives blob(node) and anc(node) (the pointer
// in use, kNoNode above the root), Act yields the active primitives in
// increasing address order, Eval supplies the value type V and prim / op /
// single / none.  The host instantiates it symbolically (tests); the device
// ablation tracer instantiates it with field values.
#pragma once

#include "st_common.h"

namespace st {

template <bool Fast, int SS, class Tree, class Act, class Eval>
HD typename Eval::V sparse_traverse(const Tree& tr, Act& act, Eval& ev, uint32_t& visited, bool& overflow) {
    using V = typename Eval::V;
    V sval[SS];
    uint32_t sanc[SS];
    int sp = 0;
    uint32_t cur = 0, nxt = 0;
    if (!act.next(cur)) return ev.none();
    bool has_next = act.next(nxt);
    while (true) {
        V val = ev.prim(cur);
        uint32_t anc = tr.anc(cur);
        if (Fast && sp > 0 && sanc[sp - 1] < anc) anc = sanc[sp - 1];
        while (true) {
            // stop (stack the value) when the next ancestor lies after the
            // next active primitive; after the last one, at the root
            if (anc == kNoNode || (has_next && anc > nxt)) break;
            const uint32_t op = anc;
            const uint32_t ob = tr.blob(op);
            const bool from_left = blob_left(tr.blob(cur));
            bool pop = false;
            if (sp > 0) {
                pop = op == sanc[sp - 1];
                if (Fast && !pop) {
                    const uint32_t oa = tr.anc(op);
                    pop = oa >= sanc[sp - 1] && (oa == kNoNode || blob_left(ob));
                }
            }
            if (pop) {
                val = ev.op(op, sval[sp - 1], val);
                sp--;
            } else {
                val = ev.single(op, val, from_left);
            }
            visited++;
            cur = op;
            anc = tr.anc(op);
            if (Fast && sp > 0 && sanc[sp - 1] < anc) anc = sanc[sp - 1];
        }
        if (sp >= SS) {
            overflow = true;
            return ev.none();
        }
        sval[sp] = val;
        sanc[sp] = anc;
        sp++;
        if (!has_next) break;
        cur = nxt;
        has_next = act.next(nxt);
    }
    if (sp != 1) overflow = true;
    return sval[0];
}

// op_type of an operator reached by one operand (Section 9): true when the
// operand passes through, false when the branch is unused
HD bool single_passes(uint32_t op_blob, bool from_left) {
    const uint32_t b = from_left ? 2u : 1u;
    return ((~b & blob_ignore(op_blob)) & 3u) == 0u;
}

// Fast ancestor pointer of node p (kNoNode for the root), from the node
// bitfields of a post-order tree.
inline uint32_t fast_ancestor(const uint32_t* blob, uint32_t p) {
    const bool d = blob_left(blob[p]);
    uint32_t a = blob_anc(blob[p]);
    while (a != kNoNode) {
        const uint32_t ab = blob[a];
        const uint32_t im = blob_ignore(ab);
        if (d ? (im & 1u) : (im & 2u)) break;   // a discards a lone operand from this side: stop there
        const uint32_t aa = blob_anc(ab);
        if (aa == kNoNode || blob_left(ab) != d) break;
        a = aa;
    }
    return a;
}

}  // namespace st
