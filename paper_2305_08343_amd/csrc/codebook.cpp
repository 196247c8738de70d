// Compression-LUT (codebook) selection on the host (Sect. 3.2.2).
//
// The paper ranks object masks by the importance SA(N) * O_m(N) / R^3 taken
// from its masked SAH (Eq. 2) and keeps the most important ones. Here:
//  - importance per child slot in float64: (SA * popcount) / R^3 with
//    SA = 2((dx*dy + dy*dz) + dz*dx) of the slot's float32 box;
//  - equal patterns add their importances in ascending slot order;
//  - the K-1 most important patterns other than the full mask are kept
//    (importance descending, ties by value ascending), then the full mask,
//    then copies of the full mask up to K entries, so every mask has a
//    conservative replacement;
//  - the codebook is sorted by (set bits ascending, value ascending), which
//    makes the lowest conservative index the tightest one (Sect. 3.2.3).
// "Value" reads a mask as an unsigned integer whose last word is the most
// significant.
#include <algorithm>
#include <array>
#include <cstring>
#include <unordered_map>

#include "internal.h"

namespace sc {
namespace {

using Mask = std::array<uint64_t, 4>;

struct MaskHash {
    size_t operator()(const Mask& m) const {
        uint64_t h = 0x9E3779B97F4A7C15ull;
        for (uint64_t w : m) {
            h ^= w + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
            h *= 0xBF58476D1CE4E5B9ull;
        }
        return (size_t)(h ^ (h >> 31));
    }
};

bool value_less(const Mask& a, const Mask& b) {
    for (int w = 3; w >= 0; --w)
        if (a[w] != b[w]) return a[w] < b[w];
    return false;
}

int popcount(const Mask& m) {
    int c = 0;
    for (uint64_t w : m) c += __builtin_popcountll(w);
    return c;
}

}  // namespace

void select_codebook(const uint64_t* masks, const float* slot_boxes, size_t S, uint32_t R,
                     uint32_t K, std::vector<uint64_t>& cb) {
    const uint32_t W = words_for(R);
    const uint32_t R3 = R * R * R;
    Mask full{};
    for (uint32_t b = 0; b < R3; ++b) full[b >> 6] |= 1ull << (b & 63);

    // first-seen order keeps the map iteration irrelevant; sums run in slot order
    std::unordered_map<Mask, size_t, MaskHash> where;
    std::vector<Mask> pattern;
    std::vector<double> importance;
    where.reserve(S / 2 + 16);
    for (size_t s = 0; s < S; ++s) {
        Mask m{};
        for (uint32_t w = 0; w < W; ++w) m[w] = masks[s * W + w];
        const float* bx = slot_boxes + 6 * s;
        const double dx = (double)bx[3] - (double)bx[0];
        const double dy = (double)bx[4] - (double)bx[1];
        const double dz = (double)bx[5] - (double)bx[2];
        const double sa = 2.0 * ((dx * dy + dy * dz) + dz * dx);
        const double imp = (sa * (double)popcount(m)) / (double)R3;
        auto it = where.find(m);
        if (it == where.end()) {
            where.emplace(m, pattern.size());
            pattern.push_back(m);
            importance.push_back(imp);
        } else {
            importance[it->second] += imp;
        }
    }
    std::vector<size_t> order;
    order.reserve(pattern.size());
    for (size_t i = 0; i < pattern.size(); ++i)
        if (pattern[i] != full) order.push_back(i);
    const size_t take = std::min<size_t>(order.size(), K - 1);
    auto more_important = [&](size_t a, size_t b) {
        if (importance[a] != importance[b]) return importance[a] > importance[b];
        return value_less(pattern[a], pattern[b]);
    };
    std::partial_sort(order.begin(), order.begin() + take, order.end(), more_important);
    std::vector<Mask> chosen;
    chosen.reserve(K);
    for (size_t i = 0; i < take; ++i) chosen.push_back(pattern[order[i]]);
    while (chosen.size() < K) chosen.push_back(full);
    std::sort(chosen.begin(), chosen.end(), [](const Mask& a, const Mask& b) {
        const int pa = popcount(a), pb = popcount(b);
        if (pa != pb) return pa < pb;
        return value_less(a, b);
    });
    cb.assign((size_t)K * W, 0);
    for (uint32_t k = 0; k < K; ++k)
        for (uint32_t w = 0; w < W; ++w) cb[(size_t)k * W + w] = chosen[k][w];
}

}  // namespace sc
