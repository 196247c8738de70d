// Collapse of the binary BVH into a 4-wide one (Sect. 3.2.4 packs four child
// boxes and their masks into one node). A 4-wide node starts from the two
// children of a binary inner node; while it has fewer than four children and
// one of them is a binary inner node, that inner child with the largest
// surface area (float64; the earliest in child order on ties) is replaced in
// place by its own two children. Nodes are numbered in DFS pre-order.
#include <cstring>

#include "internal.h"

namespace sc {
namespace {

struct Collapser {
    const HostBVH& B;
    HostBVH4& out;

    double area(uint32_t slot) const {
        const float* b = &B.cbox[6 * (size_t)slot];
        const double dx = (double)b[3] - (double)b[0];
        const double dy = (double)b[4] - (double)b[1];
        const double dz = (double)b[5] - (double)b[2];
        return 2.0 * ((dx * dy + dy * dz) + dz * dx);
    }

    // Builds the 4-wide node grown from binary inner node `node2`; `above` is
    // the number of stack entries already pending on this path.
    uint32_t grow(uint32_t node2, uint32_t above) {
        const uint32_t me = out.n4++;
        out.box.resize((size_t)out.n4 * 24, 0.0f);
        out.ref.resize((size_t)out.n4 * 4, kEmptyRef);
        out.src.resize((size_t)out.n4 * 4, kEmptyRef);
        uint32_t slot[4] = {2 * node2, 2 * node2 + 1, kEmptyRef, kEmptyRef};
        int k = 2;
        while (k < 4) {
            int pick = -1;
            double best = 0.0;
            for (int i = 0; i < k; ++i) {
                if (B.cref[slot[i]] & kLeafBit) continue;
                const double a = area(slot[i]);
                if (pick < 0 || a > best) {
                    pick = i;
                    best = a;
                }
            }
            if (pick < 0) break;
            const uint32_t inner = B.cref[slot[pick]];
            for (int i = k; i > pick + 1; --i) slot[i] = slot[i - 1];
            slot[pick] = 2 * inner;
            slot[pick + 1] = 2 * inner + 1;
            ++k;
        }
        // a visit pops this node and pushes up to k - 1 siblings of the child it continues with
        const uint32_t depth_here = above + (uint32_t)(k - 1);
        if (depth_here + 1 > out.max_stack) out.max_stack = depth_here + 1;
        for (int c = 0; c < k; ++c) {
            std::memcpy(&out.box[24 * (size_t)me + 6 * (size_t)c], &B.cbox[6 * (size_t)slot[c]], 6 * sizeof(float));
            out.src[4 * (size_t)me + c] = slot[c];
            const uint32_t r = B.cref[slot[c]];
            const uint32_t child = (r & kLeafBit) ? r : grow(r, depth_here);
            out.ref[4 * (size_t)me + c] = child;
        }
        return me;
    }
};

}  // namespace

void collapse_bvh4(const HostBVH& B, HostBVH4& out) {
    out = HostBVH4{};
    if (B.n_inner == 0 || B.root == kEmptyRef || (B.root & kLeafBit)) {
        out.root = B.root;
        return;
    }
    out.box.reserve((size_t)B.n_inner * 24);
    out.ref.reserve((size_t)B.n_inner * 4);
    out.src.reserve((size_t)B.n_inner * 4);
    Collapser c{B, out};
    out.root = c.grow(B.root, 0);
}

}  // namespace sc
