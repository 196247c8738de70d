// Collapse of the binary BVH into a 4-wide one (Sect. 3.2.4 packs four child
// boxes and their masks into one node). A 4-wide node starts from the two
// children of a binary inner node; while it has fewer than four children and
// one of them is a binary inner node, that inner child with the largest
// surface area (float64; the earliest in child order on ties) is replaced in
// place by its own two children. Nodes are numbered in DFS pre-order.
#include <cmath>
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

// Child boxes as whole steps from the node's minimum corner, the child-box
// compression of compressed wide BVHs (a layout choice; the paper keeps float
// boxes). Per node and axis, over the used children: the corner is the least
// child minimum; the step 2^e starts at the smallest e in [-126, 127] for which
// 255 steps cover the extent (rounded to double) and grows while the largest
// count, decoded, falls short of the greatest child maximum; minima round down
// and maxima up to whole steps. A plane decodes as corner + q * 2^e in float32
// with one rounding (the product is exact: 8-bit q times a normal power of
// two), exactly as the traversal's fused multiply-add does. The counts taken
// from the double quotients are first guesses only -- a child plane minus a
// corner of much larger magnitude rounds in double -- so each is moved outward
// until its decoded plane contains the child's plane, and every decoded box
// contains its child's box.
namespace {

int step_exponent(double ext) {
    if (!(ext > 0.0)) return -126;
    int k = 0;
    (void)std::frexp(ext / 255.0, &k);
    int e = k < -126 ? -126 : (k > 127 ? 127 : k);
    while (e > -126 && std::ldexp(255.0, e - 1) >= ext) --e;
    while (e < 127 && std::ldexp(255.0, e) < ext) ++e;
    return e;
}

// the plane the traversal decodes from count q: one rounding of corner + q * step
inline float decode_plane(float corner, uint32_t q, float step) { return std::fma((float)q, step, corner); }

}  // namespace

void quantise_bvh4(HostBVH4& B4, std::vector<unsigned char>& nodes) {
    nodes.assign((size_t)B4.n4 * kNode4QBytes, 0);
    for (uint32_t m = 0; m < B4.n4; ++m) {
        unsigned char* np = &nodes[(size_t)m * kNode4QBytes];
        const uint32_t* ref = &B4.ref[4 * (size_t)m];
        float* box = &B4.box[24 * (size_t)m];
        float corner[3];
        uint8_t ebias[4] = {0, 0, 0, 0};
        uint8_t q[2][3][4] = {};  // [lo / hi][axis][child]
        for (int a = 0; a < 3; ++a) {
            float lo = INFINITY, hi = -INFINITY;
            for (int c = 0; c < 4; ++c) {
                if (ref[c] == kEmptyRef) continue;
                if (box[6 * c + a] < lo) lo = box[6 * c + a];
                if (box[6 * c + 3 + a] > hi) hi = box[6 * c + 3 + a];
            }
            if (lo > hi) lo = hi = 0.0f;  // no used child
            int e = step_exponent((double)hi - (double)lo);
            while (e < 127 && decode_plane(lo, 255u, std::ldexp(1.0f, e)) < hi) ++e;
            const double step = std::ldexp(1.0, e);
            const float stepf = (float)step;
            corner[a] = lo;
            ebias[a] = (uint8_t)(e + 127);
            for (int c = 0; c < 4; ++c) {
                if (ref[c] == kEmptyRef) continue;
                const float cmin = box[6 * c + a], cmax = box[6 * c + 3 + a];
                double ql = std::floor(((double)cmin - (double)lo) / step);
                double qh = std::ceil(((double)cmax - (double)lo) / step);
                ql = ql < 0.0 ? 0.0 : (ql > 255.0 ? 255.0 : ql);
                qh = qh < 0.0 ? 0.0 : (qh > 255.0 ? 255.0 : qh);
                uint32_t ul = (uint32_t)ql, uh = (uint32_t)qh;
                for (; ul > 0 && decode_plane(lo, ul, stepf) > cmin; --ul) {
                }
                for (; uh < 255 && decode_plane(lo, uh, stepf) < cmax; ++uh) {
                }
                q[0][a][c] = (uint8_t)ul;
                q[1][a][c] = (uint8_t)uh;
                box[6 * c + a] = decode_plane(lo, ul, stepf);
                box[6 * c + 3 + a] = decode_plane(lo, uh, stepf);
            }
        }
        std::memcpy(np, corner, 12);
        std::memcpy(np + 12, ebias, 4);
        std::memcpy(np + kNode4QRefs, ref, 16);
        // words 8..13: qlo.x qlo.y qlo.z qhi.x qhi.y qhi.z, child c in byte c
        for (int a = 0; a < 3; ++a) {
            std::memcpy(np + 32 + 4 * a, q[0][a], 4);
            std::memcpy(np + 44 + 4 * a, q[1][a], 4);
        }
    }
}

}  // namespace sc
