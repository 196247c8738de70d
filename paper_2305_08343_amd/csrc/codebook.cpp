// Compression-LUT (codebook) completion on the host (Sect. 3.2.2).
//
// select_codebook_device (codebook.hip) ranks the distinct object masks by the importance
// SA(N) * O_m(N) / R^3 of the paper's masked SAH (Eq. 2) and returns the up to K-1 most
// important ones other than the full mask. Here the full mask is appended, then copies of it
// up to K entries, so every mask has a conservative replacement, and the codebook is sorted by
// (set bits ascending, value ascending), which makes the lowest conservative index the tightest
// one (Sect. 3.2.3). "Value" reads a mask as an unsigned integer whose last word is the most
// significant.
#include <algorithm>
#include <array>
#include <cstring>

#include "internal.h"

namespace sc {
namespace {

using Mask = std::array<uint64_t, 4>;

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

void finish_codebook(const std::vector<uint64_t>& picked, uint32_t R, uint32_t K, std::vector<uint64_t>& cb) {
    const uint32_t W = words_for(R);
    const uint32_t R3 = R * R * R;
    Mask full{};
    for (uint32_t b = 0; b < R3; ++b) full[b >> 6] |= 1ull << (b & 63);
    std::vector<Mask> chosen;
    chosen.reserve(K);
    for (size_t i = 0; i + W <= picked.size() && chosen.size() + 1 < K; i += W) {
        Mask m{};
        for (uint32_t w = 0; w < W; ++w) m[w] = picked[i + w];
        chosen.push_back(m);
    }
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
