// Host BVH builder: binary BVH by binned SAH.
//
// The paper builds its BVH with a binned SAH builder (Sect. 4) and notes the
// culling applies to any branching factor or builder. The split cost is the
// SAH of Eq. 1; with a size-based leaf rule the two cost constants of Eq. 1
// do not change which split is cheapest, so the cost reduces to
// SA(left)*n_left + SA(right)*n_right (float64, from float32 boxes).
//
// Exact specification (the traversal kernels and the counts they report
// depend on every choice here):
//  - triangle box: min(min(v0, v1), v2) and max(max(v0, v1), v2) per axis
//    with min(a, b) = (a < b) ? a : b, max(a, b) = (a > b) ? a : b (this
//    fixes the sign of a zero); centroid (lo + hi) * 0.5f
//  - a range's box: fold of its triangle boxes in current order from
//    (+inf, -inf)
//  - leaf iff count <= leaf_max
//  - for each axis (x, y, z) whose centroid extent is positive and whose
//    scale bins / extent is finite: bin = floor((c - lo) * scale), clamped
//    to bins-1; evaluate all bins-1 boundaries; the first strict minimum in
//    (axis, boundary) order wins; empty sides are skipped
//  - no candidate: split at count/2 in current order
//  - stable partition, left child first, inner nodes numbered in DFS
//    pre-order, triangles end in leaf order
// Large right subtrees are built on other threads into fragments with local
// node numbers and appended after the left subtree, which reproduces the
// sequential numbering exactly.
#include <cmath>
#include <cstring>
#include <future>
#include <limits>
#include <system_error>
#include <thread>
#include <atomic>

#include "internal.h"

namespace sc {
namespace {

struct Item {
    float lo[3], hi[3], c[3];
    uint32_t id;
};

struct Aabb {
    float lo[3], hi[3];
    void reset() {
        for (int j = 0; j < 3; ++j) {
            lo[j] = std::numeric_limits<float>::infinity();
            hi[j] = -std::numeric_limits<float>::infinity();
        }
    }
    void grow(const float* l, const float* h) {
        for (int j = 0; j < 3; ++j) {
            lo[j] = (l[j] < lo[j]) ? l[j] : lo[j];
            hi[j] = (h[j] > hi[j]) ? h[j] : hi[j];
        }
    }
    double area() const {
        const double dx = (double)hi[0] - (double)lo[0];
        const double dy = (double)hi[1] - (double)lo[1];
        const double dz = (double)hi[2] - (double)lo[2];
        return 2.0 * ((dx * dy + dy * dz) + dz * dx);
    }
};

// Nodes of one subtree, numbered from 0 in DFS pre-order.
struct Fragment {
    uint32_t n_inner = 0;
    uint32_t depth = 0;
    std::vector<float> cbox;
    std::vector<uint32_t> cref, range;

    // Append `g` (a subtree built separately); returns its root ref renumbered.
    uint32_t append(Fragment&& g, uint32_t g_root) {
        const uint32_t off = n_inner;
        for (uint32_t& r : g.cref)
            if (!(r & kLeafBit)) r += off;
        cbox.insert(cbox.end(), g.cbox.begin(), g.cbox.end());
        cref.insert(cref.end(), g.cref.begin(), g.cref.end());
        range.insert(range.end(), g.range.begin(), g.range.end());
        n_inner += g.n_inner;
        depth = depth > g.depth ? depth : g.depth;
        return (g_root & kLeafBit) ? g_root : g_root + off;
    }
};

class Builder {
  public:
    Builder(uint32_t leaf_max, uint32_t bins, uint32_t depth_cap)
        : leaf_max_(leaf_max), bins_(bins), depth_cap_(depth_cap) {}

    std::vector<Item> items, scratch;
    std::atomic<int> status{SC_OK};
    std::atomic<int> spare_threads{0};

    uint32_t build(Fragment& F, uint32_t b, uint32_t e, uint32_t level, Aabb& box) {
        box.reset();
        for (uint32_t i = b; i < e; ++i) box.grow(items[i].lo, items[i].hi);
        const uint32_t count = e - b;
        if (count <= leaf_max_) return kLeafBit | b | ((count - 1u) << 29);
        if (level > depth_cap_) {
            status = SC_ERR_DEPTH;
            return 0;
        }
        if (level > F.depth) F.depth = level;
        const uint32_t node = F.n_inner++;
        F.range.push_back(b);
        F.range.push_back(count);
        F.cbox.resize(12 * (size_t)F.n_inner);
        F.cref.resize(2 * (size_t)F.n_inner);

        const uint32_t mid = choose_and_partition(b, e);

        Aabb lb, rb;
        uint32_t l, r;
        if (e - mid >= kParallelMin && spare_threads.fetch_sub(1) > 0) {
            Fragment G;
            auto right = std::async(std::launch::async, [&] { return build(G, mid, e, level + 1, rb); });
            l = build(F, b, mid, level + 1, lb);
            const uint32_t g_root = right.get();
            if (status != SC_OK) return 0;
            r = F.append(std::move(G), g_root);
        } else {
            l = build(F, b, mid, level + 1, lb);
            if (status != SC_OK) return 0;
            r = build(F, mid, e, level + 1, rb);
            if (status != SC_OK) return 0;
        }
        float* dst = &F.cbox[12 * (size_t)node];
        std::memcpy(dst, lb.lo, 12);
        std::memcpy(dst + 3, lb.hi, 12);
        std::memcpy(dst + 6, rb.lo, 12);
        std::memcpy(dst + 9, rb.hi, 12);
        F.cref[2 * (size_t)node] = l;
        F.cref[2 * (size_t)node + 1] = r;
        return node;
    }

  private:
    static constexpr uint32_t kParallelMin = 1u << 16;

    uint32_t bin_of(float c, float lo, float scale) const {
        const float f = (c - lo) * scale;
        if (f >= (float)(bins_ - 1)) return bins_ - 1;
        return (uint32_t)(int)f;
    }

    // Returns the split position; partitions items[b, e) stably.
    uint32_t choose_and_partition(uint32_t b, uint32_t e) {
        Aabb cb;
        cb.reset();
        for (uint32_t i = b; i < e; ++i) cb.grow(items[i].c, items[i].c);
        double best = std::numeric_limits<double>::infinity();
        int best_axis = -1;
        uint32_t best_split = 0;
        float best_scale = 0.0f;
        std::vector<uint32_t> cnt(bins_);
        std::vector<Aabb> bin_box(bins_), left(bins_);
        std::vector<uint32_t> nleft(bins_);
        std::vector<double> cost(bins_);
        for (int a = 0; a < 3; ++a) {
            if (!(cb.hi[a] > cb.lo[a])) continue;
            const float scale = (float)bins_ / (cb.hi[a] - cb.lo[a]);
            if (!std::isfinite(scale)) continue;
            for (uint32_t k = 0; k < bins_; ++k) {
                cnt[k] = 0;
                bin_box[k].reset();
            }
            for (uint32_t i = b; i < e; ++i) {
                const uint32_t k = bin_of(items[i].c[a], cb.lo[a], scale);
                ++cnt[k];
                bin_box[k].grow(items[i].lo, items[i].hi);
            }
            Aabb run;
            run.reset();
            uint32_t nrun = 0;
            for (uint32_t s = 1; s < bins_; ++s) {
                run.grow(bin_box[s - 1].lo, bin_box[s - 1].hi);
                nrun += cnt[s - 1];
                left[s] = run;
                nleft[s] = nrun;
            }
            Aabb right;
            right.reset();
            uint32_t nright = 0;
            for (uint32_t s = bins_ - 1; s >= 1; --s) {
                right.grow(bin_box[s].lo, bin_box[s].hi);
                nright += cnt[s];
                cost[s] = (nleft[s] == 0 || nright == 0)
                              ? std::numeric_limits<double>::infinity()
                              : left[s].area() * (double)nleft[s] + right.area() * (double)nright;
            }
            for (uint32_t s = 1; s < bins_; ++s) {
                if (cost[s] < best) {
                    best = cost[s];
                    best_axis = a;
                    best_split = s;
                    best_scale = scale;
                }
            }
        }
        if (best_axis < 0) return b + (e - b) / 2u;
        uint32_t w = b;
        for (uint32_t i = b; i < e; ++i)
            if (bin_of(items[i].c[best_axis], cb.lo[best_axis], best_scale) < best_split)
                scratch[w++] = items[i];
        const uint32_t mid = w;
        for (uint32_t i = b; i < e; ++i)
            if (!(bin_of(items[i].c[best_axis], cb.lo[best_axis], best_scale) < best_split))
                scratch[w++] = items[i];
        std::memcpy(&items[b], &scratch[b], sizeof(Item) * (size_t)(e - b));
        return mid;
    }

    uint32_t leaf_max_, bins_, depth_cap_;
};

}  // namespace

sc_status build_bvh(const float* tris, uint32_t n, uint32_t leaf_max, uint32_t bins,
                    uint32_t depth_cap, HostBVH& out) {
    out = HostBVH();
    if (n == 0) return SC_OK;
    try {
        Builder B(leaf_max, bins, depth_cap);
        const unsigned hw = std::thread::hardware_concurrency();
        B.spare_threads = (int)(hw > 1 ? (hw < 64 ? hw : 64) - 1 : 0);
        B.items.resize(n);
        B.scratch.resize(n);
        for (uint32_t t = 0; t < n; ++t) {
            const float* v = tris + 9 * (size_t)t;
            Item& it = B.items[t];
            for (int j = 0; j < 3; ++j) {
                // min(min(v0, v1), v2) with min(a, b) = (a < b) ? a : b
                float lo = (v[j] < v[3 + j]) ? v[j] : v[3 + j];
                lo = (lo < v[6 + j]) ? lo : v[6 + j];
                float hi = (v[j] > v[3 + j]) ? v[j] : v[3 + j];
                hi = (hi > v[6 + j]) ? hi : v[6 + j];
                it.lo[j] = lo;
                it.hi[j] = hi;
                it.c[j] = (lo + hi) * 0.5f;
            }
            it.id = t;
        }
        Fragment F;
        Aabb root_box;
        const uint32_t root = B.build(F, 0, n, 1, root_box);
        if (B.status != SC_OK) {
            out = HostBVH();
            return (sc_status)B.status.load();
        }
        out.n_inner = F.n_inner;
        out.depth = F.depth;
        out.root = root;
        out.cbox = std::move(F.cbox);
        out.cref = std::move(F.cref);
        out.range = std::move(F.range);
        out.perm.resize(n);
        for (uint32_t i = 0; i < n; ++i) out.perm[i] = B.items[i].id;
    } catch (const std::bad_alloc&) {
        out = HostBVH();
        return SC_ERR_OOM;
    } catch (const std::system_error&) {
        out = HostBVH();
        return SC_ERR_OOM;
    }
    return SC_OK;
}

}  // namespace sc
