// C ABI of libsubcull (include/subcull.h): contexts, scene builds, traces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <limits>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

using namespace sc;

struct sc_ctx {
    int device = 0;
    sc_allocator alloc{};
    bool has_alloc = false;
    uint64_t* lut[7] = {nullptr};       // full ray-mask LUT per resolution, built on first use
    uint64_t* patterns[7] = {nullptr};  // its displacement patterns (what the traversal reads)
    std::mutex lut_mu;
    uint32_t* counters = nullptr;           // kQueueRing ray-queue counters
    std::atomic<uint32_t> next_counter{0};
    sc_tune tune{256, 8, 1, kQueueParts, 0, 0, 0, 16, 16};
    bool checks = false;                    // traces run the instances with device checks
    uint32_t* chk_flags = nullptr;          // their failed-check bits (device word)
    uint32_t chk_stack = 0, chk_nodes = 0, chk_tris = 0;  // lowered limits (0 = the scene's own)
};

struct sc_scene {
    sc_ctx* ctx = nullptr;
    sc_scene_info info{};
    HostBVH bvh;                          // host copy for export
    unsigned char* nodes = nullptr;
    float* tris = nullptr;
    uint64_t* masks = nullptr;            // exact masks [2*n_inner][W]
    uint64_t* codebook = nullptr;         // LUT mode (exported order)
    uint16_t* cidx = nullptr;             // LUT mode (exported order)
    // LUT mode, traversal copies: the tested entries re-ordered by how often a test is expected to read
    // them (the surface area of the slots using them), so the ones most read share the first cache
    // line of every bit-table row; the nodes hold these indices, and trace_order[k] is the position of
    // exported entry k
    uint64_t* codebook_trace = nullptr;
    uint16_t* cidx_trace = nullptr;
    std::vector<uint32_t> trace_order;
    uint32_t full_start = 0;              // LUT mode: first untested codebook entry (the full one by default)
    uint64_t* side_masks = nullptr;       // SPARSE mode
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // vertex bounds (ray ordering keys)
    uint32_t stride2 = kNodeBytes;        // stride of the binary node array `nodes`
    HostBVH4 bvh4;                        // 4-wide scenes: host copy for export
    unsigned char* nodes4 = nullptr;      // 4-wide nodes (kNode4Bytes, or kNode4QBytes when quantised)
    uint32_t quant4 = 0;                  // 4-wide: quantised child boxes
    uint64_t* masks4 = nullptr;           // 4-wide RAW: child masks [4*n4][W]
    uint32_t* src4 = nullptr;             // 4-wide: binary slot of each child [4*n4]
    uint32_t* bit_table = nullptr;        // LUT mode: 2-D bit table [R^3 (R^3 + 1) / 2 cell pairs][K/32]
    std::vector<std::pair<void*, size_t>> owned;
};

namespace {

thread_local std::string g_error;

sc_status fail(sc_status s, const std::string& msg) {
    g_error = msg;
    return s;
}

// a HIP error as a status: memory the runtime could not provide is SC_ERR_OOM
sc_status hip_status(hipError_t e) { return e == hipErrorOutOfMemory ? SC_ERR_OOM : SC_ERR_HIP; }

sc_status hip_fail(hipError_t e, const char* what) {
    return fail(hip_status(e), std::string(what) + ": " + hipGetErrorString(e));
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void* dev_alloc(sc_ctx* ctx, size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 256;
    if (ctx->has_alloc) return ctx->alloc.alloc(bytes, (void*)s, ctx->alloc.user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(sc_ctx* ctx, void* p, size_t bytes, hipStream_t s) {
    if (!p) return;
    if (ctx->has_alloc) ctx->alloc.free(p, bytes, (void*)s, ctx->alloc.user);
    else (void)hipFree(p);
}

// Device allocation owned by a scene.
template <typename T>
T* scene_alloc(sc_scene* sc, size_t bytes, hipStream_t s) {
    void* p = dev_alloc(sc->ctx, bytes, s);
    if (p) {
        sc->owned.emplace_back(p, bytes);
        sc->info.device_bytes += bytes;
    }
    return static_cast<T*>(p);
}

// Traversal order of a LUT scene's tested codebook entries [0, full_start): by the summed surface
// area of the slots the traversal tests that use each entry (how often a test reads it, for rays
// spread over the scene), largest first, ties by exported index; the untested tail keeps its place.
// Fills codebook_trace, cidx_trace and trace_order; waits for the stream (host temporaries).
hipError_t order_codebook_for_trace(sc_scene* sc, const std::vector<uint64_t>& cb, uint32_t S, uint32_t W,
                                    uint32_t K, uint32_t width, hipStream_t s) {
    std::vector<uint16_t> hc(S);
    hipError_t e = S ? hipMemcpyAsync(hc.data(), sc->cidx, (size_t)S * 2, hipMemcpyDeviceToHost, s) : hipSuccess;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    std::vector<double> weight(K, 0.0);
    auto add = [&](uint32_t slot) {
        const float* b = &sc->bvh.cbox[6 * (size_t)slot];
        const double dx = (double)b[3] - b[0], dy = (double)b[4] - b[1], dz = (double)b[5] - b[2];
        weight[hc[slot]] += 2.0 * ((dx * dy + dy * dz) + dz * dx);
    };
    if (width == 4) {  // the binary slots the 4-wide nodes' children came from
        const HostBVH4& B4 = sc->bvh4;
        for (size_t k = 0; k < B4.ref.size(); ++k)
            if (B4.ref[k] != kEmptyRef) add(B4.src[k]);
    } else {
        for (uint32_t q = 0; q < S; ++q) add(q);
    }
    const uint32_t F = sc->full_start;
    std::vector<uint32_t> by(F);
    for (uint32_t k = 0; k < F; ++k) by[k] = k;
    std::stable_sort(by.begin(), by.end(), [&](uint32_t a, uint32_t b) { return weight[a] > weight[b]; });
    sc->trace_order.assign(K, 0);
    for (uint32_t i = 0; i < F; ++i) sc->trace_order[by[i]] = i;
    for (uint32_t k = F; k < K; ++k) sc->trace_order[k] = k;
    std::vector<uint64_t> cbt(cb.size());
    for (uint32_t k = 0; k < K; ++k)
        std::memcpy(&cbt[(size_t)sc->trace_order[k] * W], &cb[(size_t)k * W], (size_t)W * 8);
    for (auto& c : hc) c = (uint16_t)sc->trace_order[c];
    sc->codebook_trace = scene_alloc<uint64_t>(sc, cbt.size() * 8, s);
    sc->cidx_trace = scene_alloc<uint16_t>(sc, (size_t)(S ? S : 1) * 2, s);
    if (!sc->codebook_trace || !sc->cidx_trace) return hipErrorOutOfMemory;
    e = hipMemcpyAsync(sc->codebook_trace, cbt.data(), cbt.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && S) e = hipMemcpyAsync(sc->cidx_trace, hc.data(), (size_t)S * 2, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

void scene_free_all(sc_scene* sc, hipStream_t s) {
    for (auto& pb : sc->owned) dev_free(sc->ctx, pb.first, pb.second, s);
    sc->owned.clear();
}

sc_status use_device(int dev) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(SC_ERR_NO_DEVICE, "no HIP device");
    if (cur != dev) {
        const hipError_t e = hipSetDevice(dev);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    }
    return SC_OK;
}

size_t lut_bytes(uint32_t R) { return (size_t)R * R * R * R * R * R * words_for(R) * 8; }
size_t pattern_bytes(uint32_t R) { return pattern_count(R) * words_for(R) * 8; }

// Ray-mask patterns and the full LUT of resolution R, built once per context.
sc_status ensure_lut(sc_ctx* ctx, uint32_t R, hipStream_t s) {
    std::lock_guard<std::mutex> g(ctx->lut_mu);
    if (ctx->lut[R]) return SC_OK;
    auto* pat = static_cast<uint64_t*>(dev_alloc(ctx, pattern_bytes(R), s));
    auto* lut = static_cast<uint64_t*>(dev_alloc(ctx, lut_bytes(R), s));
    if (!pat || !lut) {
        dev_free(ctx, pat, pattern_bytes(R), s);
        dev_free(ctx, lut, lut_bytes(R), s);
        return fail(SC_ERR_OOM, "ray-mask table allocation failed");
    }
    hipError_t e = launch_raymask_patterns(R, pat, s);
    if (e == hipSuccess) e = launch_raymask_lut(R, pat, lut, s);
    // finished before the tables are published: a trace on another stream may use them next
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        dev_free(ctx, pat, pattern_bytes(R), s);
        dev_free(ctx, lut, lut_bytes(R), s);
        return hip_fail(e, "ray-mask table kernels");
    }
    ctx->patterns[R] = pat;
    ctx->lut[R] = lut;
    return SC_OK;
}

bool check_params(const sc_build_params& p, std::string& why) {
    if (p.R != 4 && p.R != 6) { why = "R must be 4 or 6"; return false; }
    if (p.leaf_max < 1 || p.leaf_max > 4) { why = "leaf_max must be 1..4"; return false; }
    if (p.sah_bins < 2 || p.sah_bins > 256) { why = "sah_bins must be 2..256"; return false; }
    if (p.depth_cap < 1 || p.depth_cap > kMaxDepth) { why = "depth_cap must be 1..64"; return false; }
    if (p.mode > SC_MASK_SPARSE) { why = "unknown mask mode"; return false; }
    if (p.mode == SC_MASK_LUT && (p.codebook_size < 64 || p.codebook_size > 4096 || p.codebook_size % 64)) {
        why = "codebook_size must be a multiple of 64 in [64, 4096]";
        return false;
    }
    if (p.mode == SC_MASK_SPARSE && !p.mask_placement) { why = "SPARSE needs mask_placement"; return false; }
    if (p.width != 2 && p.width != 4) { why = "width must be 2 or 4"; return false; }
    if (p.approx_levels > 64) { why = "approx_levels must be 0..64"; return false; }
    if (p.mask_slots > 1) { why = "mask_slots must be 0 or 1"; return false; }
    if (p.bit_table > 1 || (p.bit_table && p.mode != SC_MASK_LUT)) { why = "bit_table needs LUT mode"; return false; }
    if (p.width == 4 && p.mode == SC_MASK_SPARSE) { why = "SPARSE needs width 2"; return false; }
    if (p.quantise > 1 || (p.quantise && p.width != 4)) { why = "quantise needs width 4"; return false; }
    if (p.mask_test_max >= p.R * p.R * p.R) { why = "mask_test_max must be below R^3"; return false; }
    if (p.mask_test_max && p.mode != SC_MASK_RAW && p.mode != SC_MASK_LUT) {
        why = "mask_test_max needs RAW or LUT mode";
        return false;
    }
    if (!std::isfinite(p.delta) || !std::isfinite(p.origin_bound)) { why = "non-finite delta/origin_bound"; return false; }
    return true;
}

}  // namespace

extern "C" {

void sc_build_params_default(sc_build_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->R = 6;
    p->leaf_max = 4;
    p->sah_bins = 32;
    p->depth_cap = kMaxDepth;
    p->mode = SC_MASK_RAW;
    p->codebook_size = 4096;
    p->delta = 0.0f;
    p->origin_bound = 0.0f;
    p->width = 2;
}

const char* sc_status_string(sc_status s) {
    switch (s) {
        case SC_OK: return "ok";
        case SC_ERR_INVALID_ARG: return "invalid argument";
        case SC_ERR_NO_DEVICE: return "no device";
        case SC_ERR_OOM: return "out of memory";
        case SC_ERR_DEPTH: return "BVH depth cap exceeded";
        case SC_ERR_HIP: return "HIP error";
        case SC_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* sc_last_error(void) { return g_error.c_str(); }

sc_status sc_create(int device, const sc_allocator* alloc, sc_ctx** out) {
    if (!out) return fail(SC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(SC_ERR_INVALID_ARG, "allocator needs alloc and free");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(SC_ERR_NO_DEVICE, "no HIP device");
    if (device < 0 || device >= count) return fail(SC_ERR_NO_DEVICE, "device ordinal out of range");
    sc_status st = use_device(device);
    if (st != SC_OK) return st;
    auto* ctx = new (std::nothrow) sc_ctx();
    if (!ctx) return fail(SC_ERR_OOM, "context allocation failed");
    ctx->device = device;
    if (alloc) {
        ctx->alloc = *alloc;
        ctx->has_alloc = true;
    }
    // the device address of this GPU's allocation-free scratch (taken once per device)
    const hipError_t se = scratch_init(device);
    if (se != hipSuccess) {
        delete ctx;
        return hip_fail(se, "scratch symbol address");
    }
    ctx->counters = static_cast<uint32_t*>(dev_alloc(ctx, kQueueRing * kQueueParts * 4, nullptr));
    if (!ctx->counters) {
        delete ctx;
        return fail(SC_ERR_OOM, "queue counter allocation failed");
    }
    *out = ctx;
    return SC_OK;
}

sc_status sc_destroy(sc_ctx* ctx) {
    if (!ctx) return SC_OK;
    (void)use_device(ctx->device);
    (void)hipDeviceSynchronize();
    for (uint32_t R = 0; R < 7; ++R) {
        if (ctx->lut[R]) dev_free(ctx, ctx->lut[R], lut_bytes(R), nullptr);
        if (ctx->patterns[R]) dev_free(ctx, ctx->patterns[R], pattern_bytes(R), nullptr);
    }
    dev_free(ctx, ctx->counters, kQueueRing * kQueueParts * 4, nullptr);
    if (ctx->chk_flags) dev_free(ctx, ctx->chk_flags, 4, nullptr);
    delete ctx;
    return SC_OK;
}

sc_status sc_scene_build(sc_ctx* ctx, const float* d_tris, uint32_t n, const sc_build_params* params,
                         void* stream, sc_scene** out) {
    if (!ctx || !params || !out) return fail(SC_ERR_INVALID_ARG, "ctx, params and out must be non-NULL");
    *out = nullptr;
    if (n > 0 && !d_tris) return fail(SC_ERR_INVALID_ARG, "d_tris is NULL");
    if (n >= (1u << 29)) return fail(SC_ERR_INVALID_ARG, "at most 2^29-1 triangles");
    std::string why;
    if (!check_params(*params, why)) return fail(SC_ERR_INVALID_ARG, why);
    if (params->width == 4 && n >= kRef4Full)
        return fail(SC_ERR_INVALID_ARG, "4-wide scenes hold at most 2^28-1 triangles");
    sc_status st = use_device(ctx->device);
    if (st != SC_OK) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const sc_build_params& P = *params;
    const uint32_t R = P.R, W = words_for(R);

    std::vector<float> host;
    try {
        host.resize(9 * (size_t)n);
    } catch (const std::bad_alloc&) {
        return fail(SC_ERR_OOM, "host triangle copy");
    }
    if (n) {
        hipError_t e = hipMemcpyAsync(host.data(), d_tris, host.size() * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "triangle download");
    }
    float M = 0.0f;
    float vlo[3] = {0, 0, 0}, vhi[3] = {0, 0, 0};
    for (size_t k = 0; k < host.size(); ++k) {
        const float x = host[k];
        if (!std::isfinite(x)) return fail(SC_ERR_INVALID_ARG, "non-finite triangle vertex");
        const float ax = std::fabs(x);
        M = (ax > M) ? ax : M;
        const int j = (int)(k % 3);
        if (k < 3 || x < vlo[j]) vlo[j] = x;
        if (k < 3 || x > vhi[j]) vhi[j] = x;
    }
    const float m1 = (M > 1.0f) ? M : 1.0f;
    const float ob = (P.origin_bound > 0.0f) ? P.origin_bound : 4.0f * m1;
    const float delta = (P.delta > 0.0f) ? P.delta : (m1 + ob) * 0x1p-16f;

    auto* sc = new (std::nothrow) sc_scene();
    if (!sc) return fail(SC_ERR_OOM, "scene allocation failed");
    sc->ctx = ctx;
    for (int j = 0; j < 3; ++j) {
        sc->lo[j] = vlo[j];
        sc->hi[j] = vhi[j];
    }
    auto bail = [&](sc_status code, const std::string& msg) {
        (void)hipStreamSynchronize(s);
        scene_free_all(sc, s);
        delete sc;
        return fail(code, msg);
    };

    auto t0 = std::chrono::steady_clock::now();
    st = build_bvh(host.data(), n, P.leaf_max, P.sah_bins, P.depth_cap, sc->bvh);
    if (st != SC_OK) {
        delete sc;
        return fail(st, st == SC_ERR_DEPTH ? "BVH deeper than depth_cap" : "BVH build failed");
    }
    const HostBVH& B = sc->bvh;
    sc->info.ms_bvh = ms_since(t0);
    sc_scene_info& I = sc->info;
    I.n_tris = n;
    I.n_inner = B.n_inner;
    I.depth = B.depth;
    I.root_ref = B.root;
    I.R = R;
    I.mode = P.mode;
    I.words = W;
    I.codebook_size = (P.mode == SC_MASK_LUT) ? P.codebook_size : 0;
    I.node_bytes = (P.mode == SC_MASK_RAW) ? kRawNodeBytes : kNodeBytes;
    I.delta = delta;
    I.origin_bound = ob;
    I.width = P.width;
    I.n_nodes = B.n_inner;
    I.approx_levels = P.approx_levels;
    I.bit_table = P.bit_table;
    // the densest mask still tested: the paper tests every mask but a full one
    const uint32_t test_max = P.mask_test_max ? P.mask_test_max : R * R * R - 1;
    I.mask_test_max = test_max;
    const uint32_t S = 2 * B.n_inner;
    if (P.mode == SC_MASK_SPARSE && P.placement_len != S)
        return bail(SC_ERR_INVALID_ARG, "mask_placement length must be 2*n_inner = " + std::to_string(S));

    // triangle records in leaf order: v0, e1 = v1 - v0, e2 = v2 - v0, id
    std::vector<float> rec(12 * (size_t)(n ? n : 1), 0.0f);
    for (uint32_t k = 0; k < n; ++k) {
        const uint32_t id = B.perm[k];
        const float* v = &host[9 * (size_t)id];
        float* r = &rec[12 * (size_t)k];
        r[0] = v[0]; r[1] = v[1]; r[2] = v[2];
        r[3] = v[3] - v[0]; r[4] = v[4] - v[1]; r[5] = v[5] - v[2];
        r[6] = v[6] - v[0]; r[7] = v[7] - v[1]; r[8] = v[8] - v[2];
        std::memcpy(&r[9], &id, 4);
    }
    // 4-wide scenes collapse here; with quantised child boxes, every binary slot
    // a 4-wide node uses takes the decoded box, so the masks, codebook
    // importances and exports built below all belong to the boxes the 4-wide
    // traversal tests (the collapse itself chose its expansions on exact boxes)
    std::vector<unsigned char> q4;
    if (P.width == 4) {
        collapse_bvh4(B, sc->bvh4);
        if (P.quantise) {
            quantise_bvh4(sc->bvh4, q4);
            sc->quant4 = 1;
            const HostBVH4& B4 = sc->bvh4;
            for (size_t k = 0; k < (size_t)B4.n4 * 4; ++k)
                if (B4.ref[k] != kEmptyRef)
                    std::memcpy(&sc->bvh.cbox[6 * (size_t)B4.src[k]], &B4.box[6 * k], 6 * sizeof(float));
        }
    }
    // nodes
    const uint32_t stride = I.node_bytes;
    sc->stride2 = stride;
    std::vector<unsigned char> nodes((size_t)stride * (B.n_inner ? B.n_inner : 1), 0);
    std::vector<uint32_t> side_of_slot;
    uint32_t n_masked = (P.mode == SC_MASK_NONE) ? 0 : S;
    if (P.mode == SC_MASK_SPARSE) {
        side_of_slot.assign(S, kNoMask);
        n_masked = 0;
        for (uint32_t q = 0; q < S; ++q)
            if (P.mask_placement[q]) side_of_slot[q] = n_masked++;
    }
    I.n_masked = n_masked;
    for (uint32_t i = 0; i < B.n_inner; ++i) {
        unsigned char* np = &nodes[(size_t)i * stride];
        std::memcpy(np, &B.cbox[12 * (size_t)i], 48);
        std::memcpy(np + 48, &B.cref[2 * (size_t)i], 8);
        uint32_t aux[2] = {0, 0};
        if (P.mode == SC_MASK_SPARSE) {
            aux[0] = side_of_slot[2 * i];
            aux[1] = side_of_slot[2 * i + 1];
        }
        std::memcpy(np + 56, aux, 8);
    }

    sc->nodes = scene_alloc<unsigned char>(sc, nodes.size(), s);
    sc->tris = scene_alloc<float>(sc, rec.size() * 4, s);
    if (!sc->nodes || !sc->tris) return bail(SC_ERR_OOM, "scene allocation failed");
    hipError_t e = hipMemcpyAsync(sc->nodes, nodes.data(), nodes.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sc->tris, rec.data(), rec.size() * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return bail(hip_status(e), std::string("scene upload: ") + hipGetErrorString(e));

    if (P.mode != SC_MASK_NONE) {
        st = ensure_lut(ctx, R, s);
        if (st != SC_OK) return bail(st, g_error);
    }
    if (P.mode != SC_MASK_NONE && B.n_inner > 0) {
        t0 = std::chrono::steady_clock::now();
        const size_t mask_bytes = (size_t)S * W * 8;
        sc->masks = scene_alloc<uint64_t>(sc, mask_bytes, s);
        auto* d_perm = static_cast<uint32_t*>(dev_alloc(ctx, (size_t)n * 4, s));
        auto* d_range = static_cast<uint32_t*>(dev_alloc(ctx, B.range.size() * 4, s));
        if (!sc->masks || !d_perm || !d_range) {
            dev_free(ctx, d_perm, (size_t)n * 4, s);
            dev_free(ctx, d_range, B.range.size() * 4, s);
            return bail(SC_ERR_OOM, "mask build allocation failed");
        }
        e = hipMemsetAsync(sc->masks, 0, mask_bytes, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_perm, B.perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_range, B.range.data(), B.range.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_object_masks(R, d_tris, d_perm, n, sc->nodes, stride, d_range, B.root, delta,
                                    P.approx_levels, sc->masks, s);
        if (e == hipSuccess && P.approx_levels > 0) {
            // fill part of the approximation, one launch per depth, deepest first
            std::vector<uint32_t> depth(B.n_inner, 0);
            uint32_t max_depth = 0;
            for (uint32_t i = 0; i < B.n_inner; ++i)
                for (int c = 0; c < 2; ++c) {
                    const uint32_t r = B.cref[2 * (size_t)i + c];
                    if (!(r & kLeafBit)) {
                        depth[r] = depth[i] + 1;
                        max_depth = std::max(max_depth, depth[r]);
                    }
                }
            std::vector<uint32_t> order, start(max_depth + 2, 0);
            for (uint32_t i = 0; i < B.n_inner; ++i) ++start[depth[i] + 1];
            for (uint32_t k = 1; k < start.size(); ++k) start[k] += start[k - 1];
            order.resize(2 * (size_t)B.n_inner);
            std::vector<uint32_t> fillp(start.begin(), start.end() - 1);
            for (uint32_t i = 0; i < B.n_inner; ++i) {
                const uint32_t at = fillp[depth[i]]++;
                order[2 * (size_t)at] = 2 * i;
                order[2 * (size_t)at + 1] = 2 * i + 1;
            }
            auto* d_order = static_cast<uint32_t*>(dev_alloc(ctx, order.size() * 4, s));
            auto* d_cbox = static_cast<float*>(dev_alloc(ctx, B.cbox.size() * 4, s));
            auto* d_cref = static_cast<uint32_t*>(dev_alloc(ctx, B.cref.size() * 4, s));
            if (!d_order || !d_cbox || !d_cref) e = hipErrorOutOfMemory;
            if (e == hipSuccess) e = hipMemcpyAsync(d_order, order.data(), order.size() * 4, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(d_cbox, B.cbox.data(), B.cbox.size() * 4, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(d_cref, B.cref.data(), B.cref.size() * 4, hipMemcpyHostToDevice, s);
            for (int64_t k = (int64_t)max_depth; k >= 0 && e == hipSuccess; --k) {
                // slots of the nodes at node depth k
                const uint32_t a = 2 * start[k], b = 2 * start[k + 1];
                e = launch_approx_fill(R, d_order + a, b - a, d_cbox, d_cref, P.approx_levels, delta, sc->masks, s);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            dev_free(ctx, d_order, order.size() * 4, s);
            dev_free(ctx, d_cbox, B.cbox.size() * 4, s);
            dev_free(ctx, d_cref, B.cref.size() * 4, s);
        }
        if (e == hipSuccess && P.mask_slots == 1)  // masks only where the child is a leaf
            e = launch_full_inner_slots(R, sc->nodes, stride, B.n_inner, sc->masks, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        dev_free(ctx, d_perm, (size_t)n * 4, s);
        dev_free(ctx, d_range, B.range.size() * 4, s);
        if (e != hipSuccess) return bail(hip_status(e), std::string("object masks: ") + hipGetErrorString(e));
        I.ms_masks = ms_since(t0);

        if (P.mode == SC_MASK_RAW) {
            e = launch_pack_raw(R, sc->masks, B.n_inner, test_max, sc->nodes, s);
            if (e != hipSuccess) return bail(hip_status(e), std::string("pack: ") + hipGetErrorString(e));
        } else {
            if (P.mode == SC_MASK_LUT) {
                const uint32_t K = P.codebook_size;
                t0 = std::chrono::steady_clock::now();
                std::vector<uint64_t> cb, chosen;
                const size_t ws_bytes = codebook_workspace_bytes(S, R, K);
                void* ws = dev_alloc(ctx, ws_bytes, s);
                if (!ws) return bail(SC_ERR_OOM, "codebook workspace");
                e = select_codebook_device(sc->nodes, stride, sc->masks, S, R, K, ws, chosen, s);
                dev_free(ctx, ws, ws_bytes, s);
                if (e != hipSuccess) return bail(hip_status(e), std::string("codebook: ") + hipGetErrorString(e));
                finish_codebook(chosen, R, K, cb);
                // entries are sorted by set bits: the first one denser than test_max (the full
                // mask by default) starts the untested ones
                sc->full_start = K;
                for (uint32_t k = 0; k < K; ++k) {
                    uint32_t pc = 0;
                    for (uint32_t w = 0; w < W; ++w) pc += (uint32_t)__builtin_popcountll(cb[(size_t)k * W + w]);
                    if (pc > test_max) {
                        sc->full_start = k;
                        break;
                    }
                }
                I.ms_codebook = ms_since(t0);
                t0 = std::chrono::steady_clock::now();
                const uint32_t nch = (R * R * R + 7) / 8;
                const size_t req_bytes = (size_t)nch * 256 * (K / 64) * 8;
                sc->codebook = scene_alloc<uint64_t>(sc, cb.size() * 8, s);
                sc->cidx = scene_alloc<uint16_t>(sc, (size_t)S * 2, s);
                auto* d_req = static_cast<uint64_t*>(dev_alloc(ctx, req_bytes, s));
                if (!sc->codebook || !sc->cidx || !d_req) {
                    dev_free(ctx, d_req, req_bytes, s);
                    return bail(SC_ERR_OOM, "codebook allocation failed");
                }
                e = hipMemcpyAsync(sc->codebook, cb.data(), cb.size() * 8, hipMemcpyHostToDevice, s);
                if (e == hipSuccess) e = launch_req_luts(R, sc->codebook, K, d_req, s);
                if (e == hipSuccess) e = launch_compress(R, sc->masks, S, d_req, K, sc->cidx, s);
                if (e == hipSuccess) e = order_codebook_for_trace(sc, cb, S, W, K, P.width, s);
                if (e == hipSuccess) e = launch_pack_lut(sc->cidx_trace, B.n_inner, sc->nodes, s);
                if (e == hipSuccess && P.bit_table) {
                    const size_t tb = (size_t)bit_table_rows(R) * (K / 32) * 4;
                    sc->bit_table = scene_alloc<uint32_t>(sc, tb, s);
                    if (!sc->bit_table) {
                        dev_free(ctx, d_req, req_bytes, s);
                        return bail(SC_ERR_OOM, "bit table allocation failed");
                    }
                    e = launch_bit_table(R, ctx->lut[R], sc->codebook_trace, K, sc->bit_table, s);
                }
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                dev_free(ctx, d_req, req_bytes, s);
                if (e != hipSuccess) return bail(hip_status(e), std::string("compression: ") + hipGetErrorString(e));
                I.ms_compress = ms_since(t0);
            } else {  // SPARSE: gather the placed masks (a full mask counts as none)
                std::vector<uint64_t> hmasks((size_t)S * W);
                e = hipMemcpyAsync(hmasks.data(), sc->masks, mask_bytes, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return bail(hip_status(e), std::string("mask download: ") + hipGetErrorString(e));
                n_masked = 0;
                for (uint32_t q = 0; q < S; ++q) {
                    if (side_of_slot[q] == kNoMask) continue;
                    uint32_t pc = 0;
                    for (uint32_t w = 0; w < W; ++w) pc += (uint32_t)__builtin_popcountll(hmasks[(size_t)q * W + w]);
                    side_of_slot[q] = (pc == R * R * R) ? kNoMask : n_masked++;
                }
                I.n_masked = n_masked;
                std::vector<uint64_t> side((size_t)(n_masked ? n_masked : 1) * W, 0);
                for (uint32_t i = 0; i < B.n_inner; ++i)
                    std::memcpy(nodes.data() + (size_t)i * stride + 56, &side_of_slot[2 * (size_t)i], 8);
                e = hipMemcpyAsync(sc->nodes, nodes.data(), nodes.size(), hipMemcpyHostToDevice, s);
                if (e != hipSuccess) return bail(hip_status(e), std::string("node upload: ") + hipGetErrorString(e));
                for (uint32_t q = 0; q < S; ++q)
                    if (side_of_slot[q] != kNoMask)
                        std::memcpy(&side[(size_t)side_of_slot[q] * W], &hmasks[(size_t)q * W], W * 8);
                sc->side_masks = scene_alloc<uint64_t>(sc, side.size() * 8, s);
                if (!sc->side_masks) return bail(SC_ERR_OOM, "sparse mask allocation failed");
                e = hipMemcpyAsync(sc->side_masks, side.data(), side.size() * 8, hipMemcpyHostToDevice, s);
                if (e != hipSuccess) return bail(hip_status(e), std::string("sparse upload: ") + hipGetErrorString(e));
            }
        }
    }
    if (P.width == 4) {
        const HostBVH4& B4 = sc->bvh4;
        if (B4.max_stack > kMaxStack4) return bail(SC_ERR_DEPTH, "4-wide traversal stack deeper than 128 entries");
        I.n_nodes = B4.n4;
        I.node_bytes = sc->quant4 ? kNode4QBytes : kNode4Bytes;
        if (B4.n4 > 0) {
            std::vector<unsigned char> n4;
            if (sc->quant4) {
                n4.swap(q4);
            } else {
                n4.assign((size_t)B4.n4 * kNode4Bytes, 0);
                for (uint32_t m = 0; m < B4.n4; ++m) {
                    float* f = reinterpret_cast<float*>(&n4[(size_t)m * kNode4Bytes]);
                    for (int c = 0; c < 4; ++c)
                        for (int j = 0; j < 6; ++j) f[4 * j + c] = B4.box[24 * (size_t)m + 6 * c + j];
                    std::memcpy(&n4[(size_t)m * kNode4Bytes + 96], &B4.ref[4 * (size_t)m], 16);
                }
            }
            sc->nodes4 = scene_alloc<unsigned char>(sc, n4.size(), s);
            sc->src4 = scene_alloc<uint32_t>(sc, B4.src.size() * 4, s);
            if (!sc->nodes4 || !sc->src4) return bail(SC_ERR_OOM, "4-wide node allocation failed");
            e = hipMemcpyAsync(sc->nodes4, n4.data(), n4.size(), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(sc->src4, B4.src.data(), B4.src.size() * 4, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);  // n4 is a host temporary
            if (e != hipSuccess) return bail(hip_status(e), std::string("4-wide upload: ") + hipGetErrorString(e));
            if (P.mode == SC_MASK_RAW) {
                sc->masks4 = scene_alloc<uint64_t>(sc, (size_t)B4.n4 * 4 * W * 8, s);
                if (!sc->masks4) return bail(SC_ERR_OOM, "4-wide mask allocation failed");
            }
            if (P.mode == SC_MASK_RAW || P.mode == SC_MASK_LUT) {
                e = launch_pack4(P.mode, R, sc->src4, B4.n4, sc->masks, sc->cidx_trace, test_max, sc->nodes4,
                                 sc->masks4, sc->quant4, s);
                if (e != hipSuccess) return bail(hip_status(e), std::string("4-wide pack: ") + hipGetErrorString(e));
            }
        }
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(hip_status(e), std::string("scene build: ") + hipGetErrorString(e));
    *out = sc;
    return SC_OK;
}

sc_status sc_bvh_build_host(const float* h_tris, uint32_t n, const sc_build_params* params,
                            sc_scene_host* out, sc_scene_info* info) {
    if (!params || !out || !info || (n > 0 && !h_tris)) return fail(SC_ERR_INVALID_ARG, "NULL argument");
    if (n > 0 && (!out->cbox || !out->cref || !out->range || !out->perm))
        return fail(SC_ERR_INVALID_ARG, "cbox, cref, range and perm are required");
    if (n >= (1u << 29)) return fail(SC_ERR_INVALID_ARG, "at most 2^29-1 triangles");
    std::string why;
    if (!check_params(*params, why)) return fail(SC_ERR_INVALID_ARG, why);
    for (size_t i = 0; i < 9 * (size_t)n; ++i)
        if (!std::isfinite(h_tris[i])) return fail(SC_ERR_INVALID_ARG, "non-finite triangle vertex");
    HostBVH B;
    const sc_status st = build_bvh(h_tris, n, params->leaf_max, params->sah_bins, params->depth_cap, B);
    if (st != SC_OK) return fail(st, st == SC_ERR_DEPTH ? "BVH deeper than depth_cap" : "BVH build failed");
    std::memset(info, 0, sizeof(*info));
    info->n_tris = n;
    info->n_inner = B.n_inner;
    info->depth = B.depth;
    info->root_ref = B.root;
    if (!B.cbox.empty()) std::memcpy(out->cbox, B.cbox.data(), B.cbox.size() * 4);
    if (!B.cref.empty()) std::memcpy(out->cref, B.cref.data(), B.cref.size() * 4);
    if (!B.range.empty()) std::memcpy(out->range, B.range.data(), B.range.size() * 4);
    if (!B.perm.empty()) std::memcpy(out->perm, B.perm.data(), B.perm.size() * 4);
    return SC_OK;
}

sc_status sc_scene_destroy(sc_scene* scene) {
    if (!scene) return SC_OK;
    (void)use_device(scene->ctx->device);
    (void)hipDeviceSynchronize();
    scene_free_all(scene, nullptr);
    delete scene;
    return SC_OK;
}

sc_status sc_scene_get_info(const sc_scene* scene, sc_scene_info* out) {
    if (!scene || !out) return fail(SC_ERR_INVALID_ARG, "scene and out must be non-NULL");
    *out = scene->info;
    return SC_OK;
}

sc_status sc_scene_export(const sc_scene* scene, sc_scene_host* out) {
    if (!scene || !out) return fail(SC_ERR_INVALID_ARG, "scene and out must be non-NULL");
    const HostBVH& B = scene->bvh;
    const sc_scene_info& I = scene->info;
    if (out->cbox && !B.cbox.empty()) std::memcpy(out->cbox, B.cbox.data(), B.cbox.size() * 4);
    if (out->cref && !B.cref.empty()) std::memcpy(out->cref, B.cref.data(), B.cref.size() * 4);
    if (out->range && !B.range.empty()) std::memcpy(out->range, B.range.data(), B.range.size() * 4);
    if (out->perm && !B.perm.empty()) std::memcpy(out->perm, B.perm.data(), B.perm.size() * 4);
    sc_status st = use_device(scene->ctx->device);
    if (st != SC_OK) return st;
    const size_t S = 2 * (size_t)I.n_inner;
    hipError_t e = hipSuccess;
    if (out->masks && scene->masks && S)
        e = hipMemcpy(out->masks, scene->masks, S * I.words * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && out->codebook && scene->codebook)
        e = hipMemcpy(out->codebook, scene->codebook, (size_t)I.codebook_size * I.words * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && out->cidx && scene->cidx && S)
        e = hipMemcpy(out->cidx, scene->cidx, S * 2, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "export");
    return SC_OK;
}

sc_status sc_scene_export_bit_table(const sc_scene* scene, uint32_t* out) {
    if (!scene || !out) return fail(SC_ERR_INVALID_ARG, "scene and out must be non-NULL");
    if (!scene->bit_table) return fail(SC_ERR_INVALID_ARG, "the scene has no bit table");
    sc_status st = use_device(scene->ctx->device);
    if (st != SC_OK) return st;
    // the device keeps one row per unordered cell pair; the export lists every ordered key
    const uint32_t R = scene->info.R, cells = R * R * R, kw = scene->info.codebook_size / 32;
    std::vector<uint32_t> rows;
    try {
        rows.resize((size_t)bit_table_rows(R) * kw);
    } catch (const std::bad_alloc&) {
        return fail(SC_ERR_OOM, "bit table export buffer");
    }
    const hipError_t e = hipMemcpy(rows.data(), scene->bit_table, rows.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "bit table export");
    // the device's columns follow the traversal order: exported entry k is column trace_order[k]
    const std::vector<uint32_t>& ord = scene->trace_order;
    const uint32_t K = scene->info.codebook_size;
    std::vector<uint32_t> row(kw);
    for (size_t r = 0; r < (size_t)bit_table_rows(R); ++r) {
        uint32_t* dev = rows.data() + r * kw;
        std::fill(row.begin(), row.end(), 0u);
        for (uint32_t k = 0; k < K; ++k)
            if ((dev[ord[k] >> 5] >> (ord[k] & 31u)) & 1u) row[k >> 5] |= 1u << (k & 31u);
        std::copy(row.begin(), row.end(), dev);
    }
    for (uint32_t fb = 0; fb < cells; ++fb)
        for (uint32_t fe = 0; fe < cells; ++fe)
            std::memcpy(out + ((size_t)fb * cells + fe) * kw, rows.data() + (size_t)bit_row(fb, fe) * kw,
                        (size_t)kw * 4);
    return SC_OK;
}

sc_status sc_scene_export4(const sc_scene* scene, float* box4, uint32_t* ref4, uint32_t* src4) {
    if (!scene) return fail(SC_ERR_INVALID_ARG, "scene is NULL");
    if (scene->info.width != 4) return fail(SC_ERR_INVALID_ARG, "not a 4-wide scene");
    const HostBVH4& B4 = scene->bvh4;
    if (box4 && !B4.box.empty()) std::memcpy(box4, B4.box.data(), B4.box.size() * 4);
    if (ref4 && !B4.ref.empty()) std::memcpy(ref4, B4.ref.data(), B4.ref.size() * 4);
    if (src4 && !B4.src.empty()) std::memcpy(src4, B4.src.data(), B4.src.size() * 4);
    return SC_OK;
}

namespace {
extern "C++" {  // C++ helpers of the C entry points (they take and return C++ types)

// The device-check fields of a launch record: the scene's node and triangle counts (a batch passes
// the largest; each descriptor carries its own) and the stack capacity of its width, each lowered
// to the context's test limit where one is set.
void set_check_limits(const sc_ctx* ctx, TraceLaunch& a, uint32_t n_nodes, uint32_t n_tris) {
    if (!ctx->checks) return;
    auto lower = [](uint32_t own, uint32_t lim) { return (lim && lim < own) ? lim : own; };
    a.chk_flags = ctx->chk_flags;
    a.chk_nodes = lower(n_nodes, ctx->chk_nodes);
    a.chk_tris = lower(n_tris, ctx->chk_tris);
    a.chk_stack = lower(trace_stack_capacity(a.width), ctx->chk_stack);
}

// The traversal launch: the checked instances when the context asks for them.
hipError_t run_trace(const sc_ctx* ctx, const TraceLaunch& a, hipStream_t s) {
    return ctx->checks ? launch_trace_checked(a, s) : launch_trace(a, s);
}

// Argument checks shared by the trace entry points (no HIP call).
sc_status check_trace_args(const sc_scene* scene, const float* d_rays, uint32_t n, uint32_t flags,
                           const sc_hit* d_hits, const uint32_t* d_extra, const uint32_t* d_slot_fp) {
    if (!scene) return fail(SC_ERR_INVALID_ARG, "scene is NULL");
    if (n > 0 && (!d_rays || !d_hits)) return fail(SC_ERR_INVALID_ARG, "d_rays and d_hits must be non-NULL");
    if (n > (1u << 31)) return fail(SC_ERR_INVALID_ARG, "at most 2^31 rays per call");
    if (flags & ~(uint32_t)(SC_TRACE_CULL | SC_TRACE_SHADOW | SC_TRACE_SORT))
        return fail(SC_ERR_INVALID_ARG, "unknown trace flag");
    if (((uintptr_t)d_rays & 15) || ((uintptr_t)d_hits & 15) || ((uintptr_t)d_extra & 7) ||
        ((uintptr_t)d_slot_fp & 3))
        return fail(SC_ERR_INVALID_ARG, "d_rays and d_hits must be 16-byte aligned, d_extra 8-byte");
    return SC_OK;
}

// The launch record of a single-scene trace in the context's launch shape (queue and ray order
// are set by the caller).
TraceLaunch trace_launch(const sc_scene* scene, const float* d_rays, uint32_t n, uint32_t flags, sc_hit* d_hits,
                         uint32_t* d_extra, uint32_t* d_slot_fp) {
    const sc_scene_info& I = scene->info;
    TraceLaunch a{};
    a.rays = d_rays;
    a.n = n;
    a.nodes = scene->nodes;
    a.tris = scene->tris;
    a.lut = (I.mode != SC_MASK_NONE) ? scene->ctx->lut[I.R] : nullptr;
    a.patterns = (I.mode != SC_MASK_NONE) ? scene->ctx->patterns[I.R] : nullptr;
    a.codebook = scene->codebook_trace;
    a.K = I.codebook_size;
    a.full_start = scene->full_start;
    a.side_masks = scene->side_masks;
    a.root = I.root_ref;
    a.R = I.R;
    a.mode = (I.n_inner == 0) ? (uint32_t)SC_MASK_NONE : I.mode;
    a.width = I.width;
    a.bit_table = scene->bit_table;
    if (I.width == 4) {
        // the 4-wide root is node 0 exactly when the binary root is node 0 (else the same leaf or empty ref)
        a.nodes = scene->nodes4;
        a.quant = scene->quant4;
        a.side_masks = scene->masks4;
        a.src4 = scene->src4;
    }
    a.flags = flags;
    a.origin_bound = I.origin_bound;
    a.hits = d_hits;
    a.extra = d_extra;
    a.slot_fp = d_slot_fp;
    if (a.mode == SC_MASK_SPARSE && I.n_masked == 0) a.mode = SC_MASK_NONE;
    const sc_ctx* ctx = scene->ctx;
    a.parts = ctx->tune.parts;
    a.chunk = ctx->tune.chunk;
    a.block = ctx->tune.block;
    a.stack = ctx->tune.stack;
    a.waves = ctx->tune.waves;
    a.cb_global = ctx->tune.codebook;
    a.gather = ctx->tune.gather;
    a.refill = ctx->tune.refill;
    set_check_limits(ctx, a, I.n_nodes, I.n_tris);
    return a;
}

}  // extern "C++"
}  // namespace

sc_status sc_trace(const sc_scene* scene, const float* d_rays, uint32_t n, uint32_t flags, sc_hit* d_hits,
                   uint32_t* d_extra, uint32_t* d_slot_fp, void* stream) {
    sc_status st = check_trace_args(scene, d_rays, n, flags, d_hits, d_extra, d_slot_fp);
    if (st != SC_OK) return st;
    if (n == 0) return SC_OK;
    st = use_device(scene->ctx->device);
    if (st != SC_OK) return st;
    TraceLaunch a = trace_launch(scene, d_rays, n, flags, d_hits, d_extra, d_slot_fp);
    sc_ctx* ctx = scene->ctx;
    a.queue = ctx->counters +
              (size_t)(ctx->next_counter.fetch_add(1, std::memory_order_relaxed) % kQueueRing) * kQueueParts;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const bool sort = (flags & SC_TRACE_SORT) || ctx->tune.sort;
    void* ws = nullptr;
    const size_t ws_bytes = sort ? ray_order_workspace_bytes(n) : 0;
    if (sort) {
        ws = dev_alloc(ctx, ws_bytes, s);
        if (!ws) return fail(SC_ERR_OOM, "ray order workspace");
        uint32_t* order = nullptr;
        const hipError_t e = launch_ray_order(d_rays, n, scene->lo, scene->hi, ws, &order, s);
        if (e != hipSuccess) {
            dev_free(ctx, ws, ws_bytes, s);
            return hip_fail(e, "ray order");
        }
        a.order = order;
    }
    const hipError_t e = run_trace(ctx, a, s);
    if (ws) dev_free(ctx, ws, ws_bytes, s);  // stream-ordered: the allocator reuses it after the trace
    if (e != hipSuccess) return hip_fail(e, "trace launch");
    return SC_OK;
}

sc_status sc_trace_noalloc(const sc_scene* scene, const float* d_rays, uint32_t n, uint32_t flags, sc_hit* d_hits,
                           uint32_t* d_extra, uint32_t* d_slot_fp, void* stream) {
    sc_status st = check_trace_args(scene, d_rays, n, flags, d_hits, d_extra, d_slot_fp);
    if (st != SC_OK) return st;
    const bool sort = (flags & SC_TRACE_SORT) || scene->ctx->tune.sort;
    if (sort && !scratch_fits_sort(n))
        return fail(SC_ERR_INVALID_ARG, "sc_trace_noalloc sorts at most " + std::to_string(kNoAllocMaxSortRays) +
                                            " rays (its fixed scratch); got " + std::to_string(n));
    if (n == 0) return SC_OK;
    st = use_device(scene->ctx->device);
    if (st != SC_OK) return st;
    void* scr = nullptr;
    size_t scr_bytes = 0;
    hipError_t e = scratch_get(scene->ctx->device, &scr, &scr_bytes);
    if (e != hipSuccess) return hip_fail(e, "no-allocation scratch");
    TraceLaunch a = trace_launch(scene, d_rays, n, flags, d_hits, d_extra, d_slot_fp);
    a.queue = static_cast<uint32_t*>(scr);  // cleared by the launch's reset kernel
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (sort) {
        uint32_t* order = nullptr;
        e = launch_ray_order(d_rays, n, scene->lo, scene->hi, static_cast<unsigned char*>(scr) + scratch_counter_bytes(),
                             &order, s);
        if (e != hipSuccess) return hip_fail(e, "ray order");
        a.order = order;
    }
    e = run_trace(scene->ctx, a, s);
    if (e != hipSuccess) return hip_fail(e, "trace launch");
    return SC_OK;
}

sc_status sc_ray_order(const sc_scene* scene, const float* d_rays, uint32_t n, uint32_t* d_order, void* stream) {
    if (!scene) return fail(SC_ERR_INVALID_ARG, "scene is NULL");
    if (n > 0 && (!d_rays || !d_order)) return fail(SC_ERR_INVALID_ARG, "d_rays and d_order must be non-NULL");
    if (n > (1u << 31)) return fail(SC_ERR_INVALID_ARG, "at most 2^31 rays per call");
    if (((uintptr_t)d_rays & 15) || ((uintptr_t)d_order & 3))
        return fail(SC_ERR_INVALID_ARG, "d_rays must be 16-byte aligned, d_order 4-byte");
    if (n == 0) return SC_OK;
    sc_status st = use_device(scene->ctx->device);
    if (st != SC_OK) return st;
    sc_ctx* ctx = scene->ctx;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t ws_bytes = ray_order_workspace_bytes(n);
    void* ws = dev_alloc(ctx, ws_bytes, s);
    if (!ws) return fail(SC_ERR_OOM, "ray order workspace");
    uint32_t* order = nullptr;
    hipError_t e = launch_ray_order(d_rays, n, scene->lo, scene->hi, ws, &order, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_order, order, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
    dev_free(ctx, ws, ws_bytes, s);
    if (e != hipSuccess) return hip_fail(e, "ray order");
    return SC_OK;
}

namespace {

// Checks a batch and fills its launch record and sorted descriptors.
sc_status prepare_batch(sc_ctx* ctx, const sc_batch_item* items, uint32_t n_items, uint32_t flags,
                        TraceLaunch& a, std::vector<BatchItem>& desc) {
    if (!ctx || !items || n_items == 0) return fail(SC_ERR_INVALID_ARG, "ctx and a non-empty item list are required");
    if (flags & ~(uint32_t)(SC_TRACE_CULL | SC_TRACE_SHADOW | SC_TRACE_SORT))
        return fail(SC_ERR_INVALID_ARG, "unsupported batch flag");
    if (((flags & SC_TRACE_SORT) || ctx->tune.sort) && n_items > kBatchSortItems)
        return fail(SC_ERR_UNSUPPORTED, "a sorted batch takes at most 256 items");
    const sc_scene* first = items[0].scene;
    if (!first) return fail(SC_ERR_INVALID_ARG, "item scene is NULL");
    uint64_t total = 0;
    std::vector<std::pair<double, uint32_t>> order;
    for (uint32_t k = 0; k < n_items; ++k) {
        const sc_batch_item& it = items[k];
        if (!it.scene || it.scene->ctx != ctx) return fail(SC_ERR_INVALID_ARG, "item scene missing or from another context");
        if (it.scene->info.mode != first->info.mode || it.scene->info.R != first->info.R)
            return fail(SC_ERR_INVALID_ARG, "all batch items need the same mask mode and R");
        if (it.scene->info.width != first->info.width || it.scene->quant4 != first->quant4)
            return fail(SC_ERR_INVALID_ARG, "all batch items need the same node width and child-box storage");
        if (it.n > 0 && (!it.d_rays || !it.d_hits)) return fail(SC_ERR_INVALID_ARG, "item rays/hits are NULL");
        if (((uintptr_t)it.d_rays & 15) || ((uintptr_t)it.d_hits & 15) || ((uintptr_t)it.d_extra & 7) ||
            ((uintptr_t)it.d_slot_fp & 3))
            return fail(SC_ERR_INVALID_ARG, "item rays/hits must be 16-byte aligned, extra 8-byte");
        total += it.n;
        // longest estimated work first: rays x log2(triangles)
        order.emplace_back(-(double)it.n * std::log2(2.0 + it.scene->info.n_tris), k);
    }
    if (total > (1ull << 31)) return fail(SC_ERR_INVALID_ARG, "at most 2^31 rays per batch");
    std::stable_sort(order.begin(), order.end());
    desc.clear();
    uint32_t begin = 0;
    for (const auto& o : order) {
        const sc_batch_item& it = items[o.second];
        const sc_scene* sc = it.scene;
        BatchItem d{};
        d.nodes = sc->info.width == 4 ? sc->nodes4 : sc->nodes;
        d.tris = sc->tris;
        d.codebook = sc->codebook_trace;
        d.side_masks = sc->info.width == 4 ? sc->masks4 : sc->side_masks;
        d.src4 = sc->src4;
        d.rays = it.d_rays;
        d.hits = it.d_hits;
        d.extra = it.d_extra;
        d.slot_fp = it.d_slot_fp;
        d.root = sc->info.root_ref;
        d.full_start = sc->full_start;
        d.ray_begin = begin;
        d.n_rays = it.n;
        d.origin_bound = sc->info.origin_bound;
        for (int j = 0; j < 3; ++j) {  // Morton keys of the origins in the scene's vertex bounds
            const float e = sc->hi[j] - sc->lo[j];
            const float q = 256.0f / e;
            d.key_lo[j] = sc->lo[j];
            d.key_scale[j] = (e > 0.0f && q < std::numeric_limits<float>::infinity()) ? q : 0.0f;
        }
        d.n_nodes = sc->info.n_nodes;
        d.n_tris = sc->info.n_tris;
        begin += it.n;
        desc.push_back(d);
    }
    const sc_scene_info& I = first->info;
    std::memset(&a, 0, sizeof(a));
    a.n = (uint32_t)total;
    a.R = I.R;
    a.mode = I.mode;
    a.flags = flags;
    a.lut = (I.mode != SC_MASK_NONE) ? ctx->lut[I.R] : nullptr;
    a.patterns = (I.mode != SC_MASK_NONE) ? ctx->patterns[I.R] : nullptr;
    a.chunk = ctx->tune.chunk;
    a.block = ctx->tune.block;
    a.stack = ctx->tune.stack;
    a.waves = ctx->tune.waves;
    a.parts = ctx->tune.parts;
    a.gather = ctx->tune.gather;
    a.refill = ctx->tune.refill;
    a.width = I.width;
    a.quant = first->quant4;
    a.K = I.codebook_size;
    a.n_items = n_items;
    // each descriptor carries its scene's counts; the record holds the lowered limits alone
    set_check_limits(ctx, a, ~0u, ~0u);
    if (I.mode != SC_MASK_NONE && !a.lut) {  // masks exist only if the LUT was built
        for (uint32_t k = 0; k < n_items; ++k)
            if (items[k].scene->info.n_inner) return fail(SC_ERR_INVALID_ARG, "scene without its ray-mask LUT");
    }
    return SC_OK;
}

}  // namespace

struct sc_batch {
    sc_ctx* ctx = nullptr;
    BatchItem* items = nullptr;
    size_t items_bytes = 0;
    uint32_t* counters = nullptr;
    void* sort_ws = nullptr;  // ray ordering workspace of a sorted batch
    size_t sort_bytes = 0;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

sc_status sc_trace_batch(sc_ctx* ctx, const sc_batch_item* items, uint32_t n_items, uint32_t flags,
                         void* stream) {
    TraceLaunch a;
    std::vector<BatchItem> desc;
    sc_status st = prepare_batch(ctx, items, n_items, flags, a, desc);
    if (st != SC_OK) return st;
    if (a.n == 0) return SC_OK;
    st = use_device(ctx->device);
    if (st != SC_OK) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = desc.size() * sizeof(BatchItem);
    auto* d = static_cast<BatchItem*>(dev_alloc(ctx, bytes, s));
    if (!d) return fail(SC_ERR_OOM, "batch descriptor allocation failed");
    hipError_t e = hipMemcpyAsync(d, desc.data(), bytes, hipMemcpyHostToDevice, s);
    a.items = d;
    a.queue = ctx->counters +
              (size_t)(ctx->next_counter.fetch_add(1, std::memory_order_relaxed) % kQueueRing) * kQueueParts;
    const bool sort = (flags & SC_TRACE_SORT) || ctx->tune.sort;
    const size_t ws_bytes = sort ? ray_order_workspace_bytes(a.n) : 0;
    void* ws = sort ? dev_alloc(ctx, ws_bytes, s) : nullptr;
    if (sort && !ws) e = hipErrorOutOfMemory;
    if (e == hipSuccess && sort) {
        uint32_t* order = nullptr;
        e = launch_batch_order(d, n_items, a.n, ws, &order, s);
        a.order = order;
    }
    if (e == hipSuccess) e = run_trace(ctx, a, s);
    // the descriptors and the ordering must outlive the launch: wait before releasing them
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (ws) dev_free(ctx, ws, ws_bytes, s);
    dev_free(ctx, d, bytes, s);
    if (e == hipErrorOutOfMemory) return fail(SC_ERR_OOM, "batch ray ordering workspace");
    return e == hipSuccess ? SC_OK : hip_fail(e, "batched trace");
}

sc_status sc_batch_create(sc_ctx* ctx, const sc_batch_item* items, uint32_t n_items, uint32_t flags,
                          sc_batch** out) {
    if (!out) return fail(SC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    TraceLaunch a;
    std::vector<BatchItem> desc;
    sc_status st = prepare_batch(ctx, items, n_items, flags, a, desc);
    if (st != SC_OK) return st;
    st = use_device(ctx->device);
    if (st != SC_OK) return st;
    auto* b = new (std::nothrow) sc_batch();
    if (!b) return fail(SC_ERR_OOM, "batch allocation failed");
    b->ctx = ctx;
    b->items_bytes = desc.size() * sizeof(BatchItem);
    b->items = static_cast<BatchItem*>(dev_alloc(ctx, b->items_bytes, nullptr));
    b->counters = static_cast<uint32_t*>(dev_alloc(ctx, kQueueParts * 4, nullptr));
    auto cleanup = [&](sc_status code, const std::string& msg) {
        sc_batch_destroy(b);
        return fail(code, msg);
    };
    if (!b->items || !b->counters) return cleanup(SC_ERR_OOM, "batch buffers");
    hipError_t e = hipMemcpy(b->items, desc.data(), b->items_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(SC_ERR_HIP, std::string("descriptor upload: ") + hipGetErrorString(e));
    a.items = b->items;
    a.queue = b->counters;
    const bool sort = ((flags & SC_TRACE_SORT) || ctx->tune.sort) && a.n > 0;
    if (sort) {
        b->sort_bytes = ray_order_workspace_bytes(a.n);
        b->sort_ws = dev_alloc(ctx, b->sort_bytes, nullptr);
        if (!b->sort_ws) return cleanup(SC_ERR_OOM, "batch ray ordering workspace");
    }
    e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(SC_ERR_HIP, std::string("stream: ") + hipGetErrorString(e));
    e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // the ordering kernels (keys of the current ray contents + radix sort) are part of the graph
        hipError_t le = hipSuccess;
        if (sort) {
            uint32_t* order = nullptr;
            le = launch_batch_order(b->items, n_items, a.n, b->sort_ws, &order, b->capture);
            a.order = order;
        }
        if (le == hipSuccess && a.n > 0) le = run_trace(ctx, a, b->capture);
        e = hipStreamEndCapture(b->capture, &b->graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return cleanup(SC_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    *out = b;
    return SC_OK;
}

sc_status sc_batch_launch(sc_batch* batch, void* stream) {
    if (!batch || !batch->exec) return fail(SC_ERR_INVALID_ARG, "batch is NULL");
    sc_status st = use_device(batch->ctx->device);
    if (st != SC_OK) return st;
    const hipError_t e = hipGraphLaunch(batch->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SC_OK : hip_fail(e, "graph launch");
}

sc_status sc_batch_destroy(sc_batch* batch) {
    if (!batch) return SC_OK;
    (void)use_device(batch->ctx->device);
    if (batch->capture) (void)hipStreamSynchronize(batch->capture);
    (void)hipDeviceSynchronize();
    if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
    if (batch->graph) (void)hipGraphDestroy(batch->graph);
    if (batch->capture) (void)hipStreamDestroy(batch->capture);
    dev_free(batch->ctx, batch->items, batch->items_bytes, nullptr);
    dev_free(batch->ctx, batch->counters, kQueueParts * 4, nullptr);
    if (batch->sort_ws) dev_free(batch->ctx, batch->sort_ws, batch->sort_bytes, nullptr);
    delete batch;
    return SC_OK;
}

sc_status sc_set_tune(sc_ctx* ctx, const sc_tune* tune) {
    if (!ctx || !tune) return fail(SC_ERR_INVALID_ARG, "ctx and tune must be non-NULL");
    if (!trace_config_supported(tune->block, tune->stack))
        return fail(SC_ERR_UNSUPPORTED, "no traversal kernel for this (block, stack) pair");
    if (tune->chunk < 1 || tune->chunk > 64) return fail(SC_ERR_INVALID_ARG, "chunk must be 1..64");
    if (tune->parts < 1 || tune->parts > kQueueParts) return fail(SC_ERR_INVALID_ARG, "parts must be 1..8");
    if (tune->waves > 8) return fail(SC_ERR_INVALID_ARG, "waves must be 0..8");
    if (tune->sort > 1) return fail(SC_ERR_INVALID_ARG, "sort must be 0 or 1");
    if (tune->codebook > 1) return fail(SC_ERR_INVALID_ARG, "codebook must be 0 or 1");
    if (tune->gather > 64) return fail(SC_ERR_INVALID_ARG, "gather must be 0..64");
    if (tune->refill > 64) return fail(SC_ERR_INVALID_ARG, "refill must be 0..64");
    ctx->tune = *tune;
    return SC_OK;
}

sc_status sc_get_tune(const sc_ctx* ctx, sc_tune* out) {
    if (!ctx || !out) return fail(SC_ERR_INVALID_ARG, "ctx and out must be non-NULL");
    *out = ctx->tune;
    return SC_OK;
}

sc_status sc_set_device_checks(sc_ctx* ctx, int on) {
    if (!ctx) return fail(SC_ERR_INVALID_ARG, "ctx is NULL");
    if (on && !ctx->chk_flags) {
        sc_status st = use_device(ctx->device);
        if (st != SC_OK) return st;
        ctx->chk_flags = static_cast<uint32_t*>(dev_alloc(ctx, 4, nullptr));
        if (!ctx->chk_flags) return fail(SC_ERR_OOM, "check word allocation failed");
        const hipError_t e = hipMemset(ctx->chk_flags, 0, 4);
        if (e != hipSuccess) return hip_fail(e, "check word");
    }
    ctx->checks = on != 0;
    return SC_OK;
}

sc_status sc_get_check_flags(sc_ctx* ctx, uint32_t* out, int reset) {
    if (!ctx || !out) return fail(SC_ERR_INVALID_ARG, "ctx and out must be non-NULL");
    *out = 0;
    if (!ctx->chk_flags) return SC_OK;
    sc_status st = use_device(ctx->device);
    if (st != SC_OK) return st;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(out, ctx->chk_flags, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && reset) e = hipMemset(ctx->chk_flags, 0, 4);
    if (e == hipSuccess && reset) e = hipDeviceSynchronize();
    return e == hipSuccess ? SC_OK : hip_fail(e, "check word");
}

sc_status sc_set_check_limits(sc_ctx* ctx, uint32_t max_stack, uint32_t max_nodes, uint32_t max_tris) {
    if (!ctx) return fail(SC_ERR_INVALID_ARG, "ctx is NULL");
    ctx->chk_stack = max_stack;
    ctx->chk_nodes = max_nodes;
    ctx->chk_tris = max_tris;
    return SC_OK;
}

sc_status sc_slot_features(const sc_scene* scene, float* d_out, void* stream) {
    if (!scene || !d_out) return fail(SC_ERR_INVALID_ARG, "scene and d_out must be non-NULL");
    const sc_scene_info& I = scene->info;
    if (I.n_inner == 0) return SC_OK;
    if (!scene->masks) return fail(SC_ERR_INVALID_ARG, "features need a scene built with masks");
    sc_status st = use_device(scene->ctx->device);
    if (st != SC_OK) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    sc_ctx* ctx = scene->ctx;
    const HostBVH& B = scene->bvh;
    std::vector<uint8_t> depth(B.n_inner, 0);
    depth[0] = 1;
    for (uint32_t i = 0; i < B.n_inner; ++i)  // DFS pre-order: parents come first
        for (int c = 0; c < 2; ++c) {
            const uint32_t r = B.cref[2 * (size_t)i + c];
            if (!(r & kLeafBit)) depth[r] = (uint8_t)(depth[i] + 1);
        }
    RootBox root{};
    for (int j = 0; j < 3; ++j) {
        root.lo[j] = std::min(B.cbox[j], B.cbox[6 + j]);
        root.hi[j] = std::max(B.cbox[3 + j], B.cbox[9 + j]);
    }
    const double* lo = root.lo;
    const double* hi = root.hi;
    root.area = 2.0 * (((hi[0] - lo[0]) * (hi[1] - lo[1]) + (hi[1] - lo[1]) * (hi[2] - lo[2])) +
                       (hi[2] - lo[2]) * (hi[0] - lo[0]));
    const uint32_t n = I.n_tris;
    const size_t pre_bytes = (size_t)n * 8, scr_bytes = scan_scratch_doubles(n, 1) * 8;
    const size_t rng_bytes = B.range.size() * 4;
    auto* d_pre = static_cast<double*>(dev_alloc(ctx, pre_bytes, s));
    auto* d_scr = static_cast<double*>(dev_alloc(ctx, scr_bytes, s));
    auto* d_rng = static_cast<uint32_t*>(dev_alloc(ctx, rng_bytes, s));
    auto* d_dep = static_cast<uint8_t*>(dev_alloc(ctx, depth.size(), s));
    hipError_t e = (d_pre && d_scr && d_rng && d_dep) ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipMemcpyAsync(d_rng, B.range.data(), rng_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_dep, depth.data(), depth.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_tri_shape(scene->tris, n, d_pre, s);
    if (e == hipSuccess) e = launch_prefix_scan(d_pre, n, 1, d_scr, s);
    if (e == hipSuccess)
        e = launch_slot_features(I.R, scene->nodes, scene->stride2, d_rng, d_dep, I.depth, scene->masks, d_pre, root,
                                 I.n_inner, d_out, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(ctx, d_pre, pre_bytes, s);
    dev_free(ctx, d_scr, scr_bytes, s);
    dev_free(ctx, d_rng, rng_bytes, s);
    dev_free(ctx, d_dep, depth.size(), s);
    if (e == hipErrorOutOfMemory) return fail(SC_ERR_OOM, "feature buffers");
    return e == hipSuccess ? SC_OK : hip_fail(e, "slot features");
}

sc_status sc_mlp_forward(sc_ctx* ctx, const float* d_params, const float* d_x, uint32_t n, float* d_y,
                         float* d_act, void* stream) {
    if (!ctx || !d_params || (n && (!d_x || !d_y))) return fail(SC_ERR_INVALID_ARG, "NULL argument");
    sc_status st = use_device(ctx->device);
    if (st != SC_OK) return st;
    const hipError_t e = launch_mlp_forward(d_params, d_x, n, d_y, d_act, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SC_OK : hip_fail(e, "mlp forward");
}

sc_status sc_mlp_backward(sc_ctx* ctx, const float* d_params, const float* d_x, const float* d_act,
                          const float* d_y, const float* d_t, uint32_t n, float* d_grad, float* d_work,
                          float* d_loss, void* stream) {
    if (!ctx || !d_params || !d_x || !d_act || !d_y || !d_t || !d_grad || !d_work || n == 0)
        return fail(SC_ERR_INVALID_ARG, "NULL argument or empty batch");
    sc_status st = use_device(ctx->device);
    if (st != SC_OK) return st;
    const hipError_t e =
        launch_mlp_backward(d_params, d_x, d_act, d_y, d_t, n, d_grad, d_work, d_loss, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SC_OK : hip_fail(e, "mlp backward");
}

sc_status sc_mlp_adam(sc_ctx* ctx, float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t step,
                      float lr, float beta1, float beta2, float eps, void* stream) {
    if (!ctx || !d_params || !d_grad || !d_m || !d_v || step == 0) return fail(SC_ERR_INVALID_ARG, "bad argument");
    sc_status st = use_device(ctx->device);
    if (st != SC_OK) return st;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    const hipError_t e = launch_adam(d_params, d_grad, d_m, d_v, lr, beta1, beta2, eps, bc1, bc2,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SC_OK : hip_fail(e, "adam");
}

sc_status sc_place_top(const float* h_scores, uint32_t n_slots, uint32_t n_place, uint8_t* h_placement) {
    if ((n_slots && (!h_scores || !h_placement)) || n_place > n_slots) return fail(SC_ERR_INVALID_ARG, "bad argument");
    std::vector<uint32_t> idx(n_slots);
    for (uint32_t i = 0; i < n_slots; ++i) idx[i] = i;
    // NaN counts as -infinity, so the order stays a strict weak order
    auto key = [&](uint32_t i) { return std::isnan(h_scores[i]) ? -std::numeric_limits<float>::infinity() : h_scores[i]; };
    auto better = [&](uint32_t a, uint32_t b) {
        const float sa = key(a), sb = key(b);
        if (sa != sb) return sa > sb;
        return a < b;
    };
    if (n_place < n_slots) std::nth_element(idx.begin(), idx.begin() + n_place, idx.end(), better);
    std::memset(h_placement, 0, n_slots);
    for (uint32_t i = 0; i < n_place; ++i) h_placement[idx[i]] = 1;
    return SC_OK;
}

sc_status sc_raymask_lut(sc_ctx* ctx, uint32_t R, uint64_t* d_out, void* stream) {
    if (!ctx || !d_out) return fail(SC_ERR_INVALID_ARG, "ctx and d_out must be non-NULL");
    if (R != 4 && R != 6) return fail(SC_ERR_INVALID_ARG, "R must be 4 or 6");
    sc_status st = use_device(ctx->device);
    if (st != SC_OK) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    st = ensure_lut(ctx, R, s);
    if (st != SC_OK) return st;
    const hipError_t e = launch_raymask_lut(R, ctx->patterns[R], d_out, s);
    return e == hipSuccess ? SC_OK : hip_fail(e, "ray-mask LUT kernel");
}

sc_status sc_compress_masks(sc_ctx* ctx, uint32_t R, const uint64_t* d_codebook, uint32_t K,
                            const uint64_t* d_masks, uint32_t n, uint16_t* d_idx, void* stream) {
    if (!ctx || !d_codebook || (n && (!d_masks || !d_idx)))
        return fail(SC_ERR_INVALID_ARG, "NULL argument");
    if (R != 4 && R != 6) return fail(SC_ERR_INVALID_ARG, "R must be 4 or 6");
    if (K < 64 || K > 4096 || K % 64) return fail(SC_ERR_INVALID_ARG, "K must be a multiple of 64 in [64, 4096]");
    sc_status st = use_device(ctx->device);
    if (st != SC_OK) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const uint32_t nch = (R * R * R + 7) / 8;
    const size_t req_bytes = (size_t)nch * 256 * (K / 64) * 8;
    auto* d_req = static_cast<uint64_t*>(dev_alloc(ctx, req_bytes, s));
    if (!d_req) return fail(SC_ERR_OOM, "requirement LUT allocation failed");
    hipError_t e = launch_req_luts(R, d_codebook, K, d_req, s);
    if (e == hipSuccess) e = launch_compress(R, d_masks, n, d_req, K, d_idx, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(ctx, d_req, req_bytes, s);
    return e == hipSuccess ? SC_OK : hip_fail(e, "compression");
}

}  // extern "C"
