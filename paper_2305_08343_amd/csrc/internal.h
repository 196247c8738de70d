// Internal declarations shared by the host code and the kernel launchers of
// libsubcull. Not part of the public ABI (include/subcull.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/subcull.h"

namespace sc {

constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kEmptyRef = 0xFFFFFFFFu;
constexpr uint32_t kNoHit = 0xFFFFFFFFu;
constexpr uint32_t kMaxDepth = 64;       // stack entries needed <= depth
constexpr uint32_t kNoMask = 0xFFFFFFFFu;

// Node layout (bytes). Every node holds its two children's boxes and refs in
// the first 64 bytes (one half of a 128-byte L2 line):
//   [0,24)  child 0 lo.xyz hi.xyz     [24,48) child 1 lo.xyz hi.xyz
//   [48,52) ref 0   [52,56) ref 1     [56,60) aux   [60,64) aux2
// aux  : LUT mode -> codebook index of child 0 | index of child 1 << 16
//        SPARSE   -> mask slot of child 0 (kNoMask = none); aux2 -> child 1
//        RAW      -> bit c set when child c's mask is full
// RAW nodes are 128 bytes: the raw masks follow at [64, 64 + 2*words*8).
constexpr uint32_t kNodeBytes = 64;
constexpr uint32_t kRawNodeBytes = 128;
constexpr uint32_t kTriBytes = 48;  // v0.xyz e1.xyz e2.xyz id pad pad

inline uint32_t words_for(uint32_t R) { return (R * R * R + 63u) / 64u; }

// The 2-D bit table is stored by unordered cell pair: its row for (b, e) equals the row for (e, b)
// (a ray mask is symmetric in its two cells), so only pairs with flat cell indices lo <= hi are
// kept, row hi * (hi + 1) / 2 + lo, with f = (x * R + y) * R + z; R^3 (R^3 + 1) / 2 rows.
template <int R>
constexpr uint32_t kBitRows = (uint32_t)(R * R * R) * (uint32_t)(R * R * R + 1) / 2u;
inline uint32_t bit_table_rows(uint32_t R) { return (R * R * R) * (R * R * R + 1u) / 2u; }

__host__ __device__ inline uint32_t bit_row(uint32_t fb, uint32_t fe) {
    const uint32_t lo = fb < fe ? fb : fe, hi = fb < fe ? fe : fb;
    return ((hi * (hi + 1u)) >> 1) + lo;
}

// -------------------------------------------------------------- host BVH
struct HostBVH {
    uint32_t n_inner = 0;
    uint32_t root = kEmptyRef;
    uint32_t depth = 0;
    std::vector<float> cbox;      // [n_inner][12]
    std::vector<uint32_t> cref;   // [n_inner][2]
    std::vector<uint32_t> range;  // [n_inner][2] first, count
    std::vector<uint32_t> perm;   // [n] original id per leaf-order position
};

// 4-wide BVH collapsed from the binary one (the node of Sect. 3.2.4 holds four
// child boxes and four child masks). Child c of node m: box[24m + 6c ..] (lo
// xyz, hi xyz), ref[4m + c] (leaf refs as in the binary BVH, inner refs =
// 4-wide node index, kEmptyRef when unused), src[4m + c] = the binary child
// slot it came from (kEmptyRef when unused). max_stack bounds the traversal
// stack (entries on a root-to-leaf path: one per pushed sibling, plus one).
struct HostBVH4 {
    uint32_t n4 = 0;
    uint32_t root = kEmptyRef;
    uint32_t max_stack = 1;
    std::vector<float> box;
    std::vector<uint32_t> ref, src;
};
void collapse_bvh4(const HostBVH& B, HostBVH4& out);
constexpr uint32_t kNode4Bytes = 128;  // SoA boxes (96 B), refs (16 B), aux (16 B)
// Quantised 4-wide node: corner lo xyz (12 B), step exponents + 127 (3 B, 1 B pad),
// refs (16 B), planes as bytes (child c in byte c) qlo.x qlo.y qlo.z qhi.x | qhi.y qhi.z,
// aux (8 B)
constexpr uint32_t kNode4QBytes = 64;
constexpr uint32_t kNode4QRefs = 16, kNode4QAux = 56;
// Writes the quantised nodes of B4 (aux zero) and replaces B4.box by the decoded boxes.
void quantise_bvh4(HostBVH4& B4, std::vector<unsigned char>& nodes);
// 4-wide RAW nodes: bit 28 of a child's ref marks a full mask, so the traversal reads
// the flags with the refs and needs no aux load. Leaf first-triangle and node indices
// of 4-wide scenes stay below 2^28 (checked at build); the traversal clears the bit
// before it uses a ref.
constexpr uint32_t kRef4Full = 1u << 28;
constexpr uint32_t kMaxStack4 = 128;   // traversal stack entries per ray for the 4-wide BVH

// Binned SAH build; returns SC_OK, SC_ERR_DEPTH or SC_ERR_OOM.
sc_status build_bvh(const float* tris, uint32_t n, uint32_t leaf_max, uint32_t bins,
                    uint32_t depth_cap, HostBVH& out);

// Codebook of K masks (Eq. 2 importance, Sect. 3.2.2) in two steps: on the device, the up to K-1
// most important distinct masks other than the full one (importance descending, ties by value
// ascending; slot s's box is child s & 1 of binary node s >> 1 in `nodes`), returned as `chosen`
// (W words each), with codebook_workspace_bytes(S, R, K) bytes of device workspace; then on the
// host, the full mask appended up to K entries and the whole sorted by set-bit count then value.
size_t codebook_workspace_bytes(uint32_t S, uint32_t R, uint32_t K);
hipError_t select_codebook_device(const unsigned char* nodes, uint32_t stride, const uint64_t* masks, uint32_t S,
                                  uint32_t R, uint32_t K, void* workspace, std::vector<uint64_t>& chosen,
                                  hipStream_t s);
void finish_codebook(const std::vector<uint64_t>& chosen, uint32_t R, uint32_t K, std::vector<uint64_t>& cb);

// ------------------------------------------------------ kernel launchers
// One scene's share of a batched launch (device-resident descriptor).
struct BatchItem {
    const unsigned char* nodes;
    const float* tris;
    const uint64_t* codebook;
    const uint64_t* side_masks;
    const float* rays;
    sc_hit* hits;
    uint32_t* extra;
    uint32_t* slot_fp;
    uint32_t root, full_start, ray_begin, n_rays;
    float origin_bound;
    uint32_t pad;
    const uint32_t* src4;  // 4-wide scenes: binary slot of child [4*node+c] (shadow counts)
    float key_lo[3];       // ray ordering: the scene's vertex bounds' minimum corner and
    float key_scale[3];    // 256 / extent per axis (0 for a flat axis)
    uint32_t n_nodes;      // device checks: the scene's inner nodes (at its width) and triangles
    uint32_t n_tris;
};
static_assert(sizeof(BatchItem) == 128, "batch descriptor layout");

struct TraceLaunch {
    const float* rays;
    uint32_t n;
    const unsigned char* nodes;
    const float* tris;          // kTriBytes records in leaf order
    const uint64_t* lut;        // full ray-mask LUT [R^6][W]
    const uint64_t* patterns;   // displacement patterns [R(2R-1)^2][W]
    const uint64_t* codebook;   // LUT mode
    uint32_t K;                 // codebook entries (LUT mode)
    uint32_t full_start;        // first codebook index holding the full mask (K if none)
    const uint64_t* side_masks; // SPARSE mode
    uint32_t root;
    uint32_t R;
    uint32_t mode;
    uint32_t flags;
    float origin_bound;
    sc_hit* hits;
    uint32_t* extra;
    uint32_t* slot_fp;
    uint32_t* queue;            // kQueueParts ray-queue counters for this launch (zeroed on the stream first)
    uint32_t parts;             // ray partitions in use, 1..kQueueParts
    uint32_t chunk;             // rays per queue fetch = 64 * chunk
    uint32_t block, stack;      // threads per block, LDS stack entries per lane
    uint32_t waves;             // cap on resident waves per SIMD, 0 = occupancy limit
    uint32_t cb_global;         // LUT mode: 1 = read the codebook from global memory even when it fits LDS
    uint32_t gather;            // leaf gathering: lanes at leaves wait while fewer than this many are (0 = off)
    uint32_t refill;            // idle lanes take rays once this many are idle or none is busy (0, 1 = at once)
    const uint32_t* order;      // single scene: rays are taken in this order (NULL = index order)
    uint32_t width;             // 2 (binary nodes) or 4 (4-wide nodes; side_masks = raw masks [4*node+c])
    uint32_t quant = 0;         // width 4: 1 = quantised child boxes (kNode4QBytes nodes, aux in the last piece)
    const uint32_t* src4;       // 4-wide: binary slot of child [4*node+c] (shadow counts)
    const uint32_t* bit_table;  // LUT mode: [R^6][K/32] ray-mask key x codebook entry bits, or NULL
    const BatchItem* items;     // batched launch: per-scene descriptors sorted by ray_begin, else null
    uint32_t n_items;
    // Device checks (the instances compiled with SC_DEVICE_CHECKS; ignored by the others): every
    // inner-node reference must be below chk_nodes, every leaf's triangle range end at or below
    // chk_tris (a batch: also below its scene's own counts), a lane hold at most chk_stack stack
    // entries, a tested codebook index be below K. A failed check sets its kChk bit in *chk_flags
    // and the access does not happen (the ray ends, or the entry is not pushed).
    uint32_t* chk_flags;
    uint32_t chk_nodes, chk_tris, chk_stack;
};

constexpr uint32_t kChkNode = SC_CHECK_NODE, kChkTri = SC_CHECK_TRI, kChkStack = SC_CHECK_STACK, kChkIndex = SC_CHECK_INDEX;

// stack entries one lane can hold (LDS + private), by node width
constexpr uint32_t trace_stack_capacity(uint32_t width) { return width == 2 ? kMaxDepth + 1 : kMaxStack4; }

// (block, stack) pairs with compiled traversal kernels.
constexpr uint32_t kTraceConfigs[][2] = {{256, 8}, {128, 8}, {256, 12}, {256, 4}, {128, 16}};
bool trace_config_supported(uint32_t block, uint32_t stack);
constexpr uint32_t kQueueRing = 1024;  // launch counter sets per context
constexpr uint32_t kQueueParts = 8;    // counters per set (one per XCD of an MI355X)

hipError_t launch_trace(const TraceLaunch& a, hipStream_t s);
// the same kernels with the device checks compiled in (kernels_trace_checked.hip)
hipError_t launch_trace_checked(const TraceLaunch& a, hipStream_t s);

// Allocation-free traces (noalloc.hip): a file-scope device array per GPU holds the queue
// counters and the sort workspace for up to kNoAllocMaxSortRays rays. scratch_init takes its
// device address once per device (the device current); scratch_get returns it and its size.
constexpr uint32_t kNoAllocMaxSortRays = 1u << 22;
hipError_t scratch_init(int device);
hipError_t scratch_get(int device, void** ptr, size_t* bytes);
size_t scratch_counter_bytes();
bool scratch_fits_sort(uint32_t n);
// ray order by Morton code of the origin in [lo, hi] (stable radix sort); *order points into workspace
size_t ray_order_workspace_bytes(uint32_t n);
// Stable LSD radix sort (8 bits a pass, from bit 0) of the n (key, value) pairs held in the first
// two n-word arrays of `workspace` (ray_order_workspace_bytes(n) bytes); returns the sorted values,
// which an even number of passes leaves in the second array.
uint32_t* sort_pairs_u32(void* workspace, uint32_t n, uint32_t passes, hipStream_t s);
// Exclusive prefix sum of a[m] in place; `sums` holds scan_u32_sums(m) words of scratch.
size_t scan_u32_sums(size_t m);
hipError_t exclusive_scan_u32(uint32_t* a, size_t m, uint32_t* sums, hipStream_t s);
hipError_t launch_ray_order(const float* rays, uint32_t n, const float lo[3], const float hi[3], void* workspace,
                            uint32_t** order, hipStream_t s);
// batched launches: the n rays of n_items (<= kBatchSortItems) descriptors (sorted by ray_begin)
// ordered by (item, Morton code of the origin in the item's key bounds); the same workspace size
constexpr uint32_t kBatchSortItems = 256;
hipError_t launch_batch_order(const BatchItem* items, uint32_t n_items, uint32_t n, void* workspace,
                              uint32_t** order, hipStream_t s);
hipError_t launch_raymask_patterns(uint32_t R, uint64_t* patterns, hipStream_t s);
hipError_t launch_raymask_lut(uint32_t R, const uint64_t* patterns, uint64_t* out, hipStream_t s);
inline size_t pattern_count(uint32_t R) { return (size_t)R * (2 * R - 1) * (2 * R - 1); }
// levels = 0: exact masks; L > 0: the triangle part of the approximation (slots at most L above the leaf)
hipError_t launch_object_masks(uint32_t R, const float* tris_orig, const uint32_t* perm, uint32_t n,
                               const unsigned char* nodes, uint32_t node_stride,
                               const uint32_t* range, uint32_t root, float delta, uint32_t levels,
                               uint64_t* masks, hipStream_t s);
// every slot whose child (ref at node bytes 48 + 4c) is an inner node gets the full mask
hipError_t launch_full_inner_slots(uint32_t R, const unsigned char* nodes, uint32_t stride, uint32_t n_inner,
                                   uint64_t* masks, hipStream_t s);
// approximation, fill part (Alg. 2) for the given slots of one depth; deeper depths first
hipError_t launch_approx_fill(uint32_t R, const uint32_t* slots, uint32_t count, const float* cbox,
                              const uint32_t* cref, uint32_t levels, float delta, uint64_t* masks, hipStream_t s);
hipError_t launch_req_luts(uint32_t R, const uint64_t* cb, uint32_t K, uint64_t* req, hipStream_t s);
hipError_t launch_compress(uint32_t R, const uint64_t* masks, uint32_t n, const uint64_t* req,
                           uint32_t K, uint16_t* idx, hipStream_t s);
// a mask with more than test_max set bits is marked untested (a full mask at test_max = R^3 - 1)
hipError_t launch_pack_raw(uint32_t R, const uint64_t* masks, uint32_t n_inner, uint32_t test_max,
                           unsigned char* nodes, hipStream_t s);
hipError_t launch_pack_lut(const uint16_t* idx, uint32_t n_inner, unsigned char* nodes, hipStream_t s);
// 2-D bit table: bit k of row key = (LUT[key] AND codebook[k]) != 0; [R^6][K/32] words
hipError_t launch_bit_table(uint32_t R, const uint64_t* lut, const uint64_t* cb, uint32_t K, uint32_t* out,
                            hipStream_t s);
// 4-wide nodes: gather each child's raw mask (and full flag) or codebook index from its binary slot
hipError_t launch_pack4(uint32_t mode, uint32_t R, const uint32_t* src4, uint32_t n4, const uint64_t* masks,
                        const uint16_t* cidx, uint32_t test_max, unsigned char* nodes4, uint64_t* masks4,
                        uint32_t quant, hipStream_t s);

// learned placement
constexpr int kMlpParams = SC_MLP_PARAMS;
// per-triangle thinness [n] (leaf order), float64
hipError_t launch_tri_shape(const float* rec, uint32_t n, double* out, hipStream_t s);
size_t scan_scratch_doubles(uint32_t n, uint32_t rows);
hipError_t launch_prefix_scan(double* a, uint32_t n, uint32_t rows, double* scratch, hipStream_t s);
// the root box (union of the root's child boxes) and its surface area, for the slot features
struct RootBox {
    double lo[3], hi[3], area;
};
hipError_t launch_slot_features(uint32_t R, const unsigned char* nodes, uint32_t stride, const uint32_t* range,
                                const uint8_t* depth, uint32_t max_depth, const uint64_t* masks,
                                const double* prefix, const RootBox& root, uint32_t n_inner, float* out,
                                hipStream_t s);
hipError_t launch_mlp_forward(const float* prm, const float* x, uint32_t n, float* y, float* act, hipStream_t s);
hipError_t launch_mlp_backward(const float* prm, const float* x, const float* act, const float* y, const float* t,
                               uint32_t n, float* grad, float* work, float* loss, hipStream_t s);
hipError_t launch_adam(float* prm, const float* grad, float* m, float* v, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t s);

}  // namespace sc
