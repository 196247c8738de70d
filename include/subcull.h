/*
 * subcull.h - C ABI of the MI355X subspace-culling ray tracer.
 *
 * Method: Yoshimura & Harada, "Subspace Culling for Ray-Box Intersection"
 * (PACMCGIT 6(1), 2023). Every BVH child box carries an R x R x R occupancy
 * bit mask (the "object mask", Sect. 3.1.1); a ray that passes the slab test
 * of the box is converted into a "ray mask" of the same grid by a lookup
 * keyed by the voxels of its entry and exit points (Alg. 1), and the child is
 * culled when the two masks share no bit (Sect. 3.1.2, Alg. 4). Masks may be
 * stored raw or as indices into a conservative codebook (Sect. 3.2.2-3.2.3,
 * Alg. 3).
 *
 * Conventions for every function:
 *  - The return value is an sc_status; no C++ exception crosses the ABI.
 *  - Argument checks happen before any HIP call, so a bad argument returns
 *    SC_ERR_INVALID_ARG on any machine; sc_last_error() then holds a
 *    thread-local message.
 *  - "device" pointers are HIP device memory (for instance a torch tensor's
 *    data_ptr); "host" pointers are ordinary memory. Callers own every buffer
 *    they pass in; a scene owns the memory it allocates.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Traces are asynchronous on that stream and never synchronise the host;
 *    scene builds synchronise (the BVH is built on the host, and the
 *    codebook's selection is read back to finish it there).
 *  - An asynchronous HIP failure is reported as SC_ERR_HIP by the call that
 *    observes it; memory that the allocator or the HIP runtime cannot provide
 *    is SC_ERR_OOM, returned before any kernel would use the missing buffer,
 *    and the call releases what it had allocated.
 */
#ifndef SUBCULL_H
#define SUBCULL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SC_OK = 0,
    SC_ERR_INVALID_ARG = 1,  /* null pointer, size or parameter out of range */
    SC_ERR_NO_DEVICE = 2,    /* no HIP device with that ordinal */
    SC_ERR_OOM = 3,          /* an allocation (device or host) failed */
    SC_ERR_DEPTH = 4,        /* the BVH would exceed depth_cap */
    SC_ERR_HIP = 5,          /* a HIP runtime call failed */
    SC_ERR_UNSUPPORTED = 6   /* valid request the library does not implement */
} sc_status;

/* How object masks are stored (Sect. 3.2.2, 3.2.4). */
typedef enum {
    SC_MASK_NONE = 0,   /* plain BVH, no culling (the baseline of Tables 1-2)  */
    SC_MASK_RAW = 1,    /* R^3 bits per child, stored in the node             */
    SC_MASK_LUT = 2,    /* 16-bit index into a K-entry conservative codebook  */
    SC_MASK_SPARSE = 3  /* raw masks on a chosen subset of child slots only    */
} sc_mask_mode;

/* sc_trace flags */
enum {
    SC_TRACE_CULL = 1u,    /* apply the mask test (else masks are ignored)        */
    SC_TRACE_SHADOW = 2u,  /* evaluate masks without culling; count would-be culls
                              per child slot into d_slot_fp                      */
    SC_TRACE_SORT = 4u     /* take the rays in the Morton order of their origins
                              (stable radix sort on the device, workspace from
                              the context allocator); results are unchanged     */
};

typedef struct sc_ctx sc_ctx;
typedef struct sc_scene sc_scene;

/* Optional device allocator. alloc returns device memory of `bytes` bytes
 * usable on `stream`, or NULL; free releases it. With no allocator the
 * library uses hipMalloc/hipFree. */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*free)(void* ptr, size_t bytes, void* stream, void* user);
    void* user;
} sc_allocator;

typedef struct {
    uint32_t R;             /* mask resolution: 4 (64 bits) or 6 (216 bits)      */
    uint32_t leaf_max;      /* triangles per leaf, 1..4 (default 4)               */
    uint32_t sah_bins;      /* SAH bins per axis, 2..256 (default 32)             */
    uint32_t depth_cap;     /* max inner nodes on a root-to-leaf path, 1..64      */
    uint32_t mode;          /* sc_mask_mode                                       */
    uint32_t codebook_size; /* K for SC_MASK_LUT: multiple of 64, 64..4096; Alg. 3
                               reads a mask in 8-bit chunks (ceil(R^3 / 8)
                               requirement tables of 256 rows), a fixed width  */
    float delta;            /* voxel dilation; <= 0 selects the default           */
    float origin_bound;     /* masks are skipped for rays with max|o| above this;
                               <= 0 selects the default                          */
    const uint8_t* mask_placement; /* SC_MASK_SPARSE: host [2*n_inner] 0/1 per child
                               slot (slot = 2*node + child); else NULL            */
    uint32_t placement_len; /* length of mask_placement                            */
    uint32_t width;         /* 2: binary BVH; 4: 4-wide BVH collapsed from it, each
                               node with four child boxes and four child masks
                               (Sect. 3.2.4); modes NONE, RAW, LUT; at most
                               2^28-1 triangles (default 2)                       */
    uint32_t approx_levels; /* 0: exact masks from every triangle below (L = inf);
                               L in 1..64: approximate masks of Sect. 3.2.1 /
                               Alg. 2 -- triangles of leaves at most L levels
                               below, plus the masks of inner nodes exactly L
                               levels below projected onto the box (each set
                               voxel fills the parent voxels its extent plus
                               2 delta covers); always a superset of the exact
                               mask                                              */
    uint32_t bit_table;     /* LUT mode: 1 builds the 2-D bit table of Sect. 3.2.2
                               (bit (key, k) = ray mask LUT[key] AND codebook
                               entry k is nonzero; a key's row equals its
                               reversed pair's, so the device keeps one row per
                               unordered cell pair: R^3 (R^3 + 1) / 2 * K / 8
                               bytes) and single
                               scene traces test a compressed mask with one bit
                               of it; results are unchanged (default 0)           */
    uint32_t mask_slots;    /* which child slots keep a testable mask: 0 = every
                               slot (default, as in the paper), 1 = only slots
                               whose child is a leaf -- slots of inner children
                               get the full mask, which is never tested, so the
                               traversal tests masks where a cull saves
                               triangle tests (results unchanged)                */
    uint32_t quantise;      /* width 4 (modes NONE, RAW, LUT): 1 stores child boxes as
                               8-bit steps from the node's minimum corner (one
                               power-of-two step per axis, the smallest whose
                               255 steps, decoded in float32, reach the node's
                               maximum; each plane moved outward until its
                               float32 decode contains the child's plane),
                               64-byte nodes. Decoded boxes contain
                               the exact ones, so hits are those of the exact
                               boxes; the binary slots the 4-wide nodes use take
                               the decoded boxes, and masks, exports and counts
                               follow them (default 0)                           */
    uint32_t mask_test_max; /* RAW and LUT modes: the most set bits a stored mask
                               (raw mask, or the codebook entry a slot points
                               to) may have and still be tested; denser masks
                               pass untested, as a full mask always does (it
                               cannot cull). Skipping a test never changes a
                               hit. 0 selects R^3 - 1 (only full masks untested,
                               the paper's method); 1..R^3 - 1 otherwise       */
} sc_build_params;

typedef struct {
    uint32_t n_tris, n_inner, depth, root_ref;
    uint32_t R, mode, codebook_size, words;  /* words = 64-bit words per mask  */
    uint32_t node_bytes;                     /* stride of one inner node (4-wide: 128, quantised 64) */
    uint32_t n_masked;                       /* slots that carry a mask         */
    uint32_t width;                          /* 2 or 4                          */
    uint32_t n_nodes;                        /* inner nodes traversed: n_inner,
                                                or 4-wide nodes when width 4    */
    uint32_t approx_levels;                  /* as built (0 = exact masks)      */
    uint32_t bit_table;                      /* 1 if the scene has a bit table  */
    uint32_t mask_test_max;                  /* as built (R^3 - 1 by default)   */
    float delta, origin_bound;
    uint64_t device_bytes;                   /* scene-owned device memory       */
    double ms_bvh, ms_masks, ms_codebook, ms_compress;  /* build phases (host clock) */
} sc_scene_info;

/* One result per ray. prim = original triangle index or 0xFFFFFFFF on a
 * miss; t = hit distance or +inf; box_tests = ray-box slab tests executed;
 * tri_tests = ray-triangle tests executed. */
typedef struct {
    uint32_t prim;
    float t;
    uint32_t box_tests;
    uint32_t tri_tests;
} sc_hit;

/* Host buffers for sc_scene_export, each sized from sc_scene_info; any
 * pointer may be NULL to skip that array. */
typedef struct {
    float* cbox;        /* [n_inner][12]: child0 lo xyz, hi xyz, child1 lo, hi   */
    uint32_t* cref;     /* [n_inner][2]: child refs (bit31 leaf: bits0-28 first
                           triangle, bits29-30 count-1; else inner node index) */
    uint32_t* range;    /* [n_inner][2]: first triangle, count of the subtree  */
    uint32_t* perm;     /* [n_tris]: original index of each leaf-order triangle */
    uint64_t* masks;    /* [2*n_inner][words]: exact object masks (RAW, LUT)    */
    uint64_t* codebook; /* [K][words] (LUT)                                      */
    uint16_t* cidx;     /* [2*n_inner] codebook index per child slot (LUT)       */
} sc_scene_host;

/* Launch shape of the traversal: threads per block, LDS stack entries per
 * lane (deeper entries spill to private memory), rays per queue fetch
 * (64 * chunk) and the number of contiguous ray partitions with their own
 * queue (waves start on partition block % parts, i.e. per XCD when parts is
 * 8, and steal from the others), and a cap on the waves resident per SIMD
 * (the persistent grid is sized to it; 0 = as many as registers and LDS
 * allow), whether traces sort their rays as with SC_TRACE_SORT (single-scene
 * and batched launches), and where LUT-mode single-scene traces read the codebook
 * (Sect. 3.2.2): 0 = a copy in LDS when it fits (K * words <= 1024 64-bit
 * words), 1 = from global memory through the caches, and leaf gathering:
 * a lane whose ray stands at a leaf waits (its ray does not advance) while
 * fewer than `gather` lanes of its wave do and another lane stands at an
 * inner node, at most gather / 2 steps in a row, so that the wave runs the
 * triangle tests for many lanes at once (0 = never wait), and refill
 * gathering: idle lanes take new rays only when at least `refill` lanes of
 * the wave are idle or none is busy (0 or 1 = as soon as one is idle).
 * Results never depend on it. Supported (block, stack) pairs: (256,8)
 * (128,8) (256,12) (256,4) (128,16); chunk 1..64; parts 1..8; waves 0..8;
 * sort 0 or 1; codebook 0 or 1; gather 0..64; refill 0..64. */
typedef struct {
    uint32_t block;
    uint32_t stack;
    uint32_t chunk;
    uint32_t parts;
    uint32_t waves;
    uint32_t sort;
    uint32_t codebook;
    uint32_t gather;
    uint32_t refill;
} sc_tune;

/* Fill `p` with the defaults: R 6, leaf_max 4, 32 bins, depth cap 64, RAW,
 * K 4096, default delta and origin bound. */
void sc_build_params_default(sc_build_params* p);

/* Create a context on HIP device `device`. `alloc` may be NULL. The context
 * caches the ray-mask LUTs and must outlive its scenes. */
sc_status sc_create(int device, const sc_allocator* alloc, sc_ctx** out);
sc_status sc_destroy(sc_ctx* ctx); /* NULL-safe */

/*
 * Build a scene from `n` triangles (device float32 [n][3][3], vertex-major).
 *  1. copies the triangles to the host and builds a binary BVH by binned SAH
 *     (the builder named in Sect. 4; split cost of Eq. 1 with a size-based
 *     leaf rule), DFS pre-order, triangles reordered into leaf order;
 *  2. builds the ray-mask LUT of resolution R (Sect. 3.1.1, Alg. 1) on the
 *     device if the context lacks it;
 *  3. (RAW, LUT, SPARSE) builds exact object masks for every child slot on
 *     the device: voxels of the child box that a descendant triangle
 *     overlaps, dilated by delta (Sect. 3.1.1, 3.2.1 with L = infinity);
 *  4. (LUT) selects the codebook by the importance SA(N) O_m(N) / R^3 of Eq. 2
 *     on the device (the K - 1 most important distinct masks; the host pads
 *     with the full mask and sorts the K entries), builds the requirement LUTs
 *     and compresses every mask with Alg. 3 on the device (Sect. 3.2.2-3.2.3);
 *  5. packs the device node array; with width 4 also collapses the BVH into
 *     4-wide nodes (see sc_scene_export4) whose children take the masks and
 *     codebook indices of the binary slots they came from.
 * Errors: SC_ERR_INVALID_ARG (null pointers, n >= 2^29, R not 4 or 6, bad
 * K, non-finite vertex, width not 2 or 4, SPARSE with width 4), SC_ERR_DEPTH
 * (also: a 4-wide traversal stack above 128 entries), SC_ERR_OOM, SC_ERR_HIP. n = 0 gives an
 * empty scene whose traces all miss. Synchronises `stream`.
 */
sc_status sc_scene_build(sc_ctx* ctx, const float* d_tris, uint32_t n, const sc_build_params* params,
                         void* stream, sc_scene** out);
sc_status sc_scene_destroy(sc_scene* scene); /* NULL-safe */

/* Step 1 of sc_scene_build alone, on the host (no device needed): the binned
 * SAH BVH of `n` host triangles (float32 [n][3][3]) under params' leaf_max,
 * sah_bins and depth_cap. out->cbox/cref/range must hold max(n,1) nodes and
 * out->perm n entries (masks, codebook, cidx are ignored). info receives
 * n_inner, depth and root_ref (other fields zero). Errors as sc_scene_build. */
sc_status sc_bvh_build_host(const float* h_tris, uint32_t n, const sc_build_params* params,
                            sc_scene_host* out, sc_scene_info* info);
sc_status sc_scene_get_info(const sc_scene* scene, sc_scene_info* out);

/* Copy the scene's BVH, masks and codebook into caller host buffers
 * (synchronous). Used to check the build against an independent reference.
 * In a scene built with quantise = 1 the child slots that 4-wide nodes use
 * hold their decoded boxes (the boxes the masks were built on). */
sc_status sc_scene_export(const sc_scene* scene, sc_scene_host* out);

/* Copy a 4-wide scene's nodes (host, synchronous): box4 float [n_nodes][4][6]
 * (child lo xyz, hi xyz; the decoded boxes when the scene was built with
 * quantise = 1), ref4 uint32 [n_nodes][4] (leaf refs as in the
 * binary BVH, inner refs = 4-wide node index, 0xFFFFFFFF = unused child),
 * src4 uint32 [n_nodes][4] (the binary child slot each child came from; its
 * mask and codebook index). The collapse: a node starts from the two children
 * of a binary inner node and, while it has fewer than four children and one
 * is a binary inner node, replaces the one with the largest surface area
 * (the earliest on ties) by its two children; DFS pre-order. Any pointer may
 * be NULL. SC_ERR_INVALID_ARG for a binary scene. */
sc_status sc_scene_export4(const sc_scene* scene, float* box4, uint32_t* ref4, uint32_t* src4);

/* Copy a LUT scene's 2-D bit table to host `out` (uint32 [R^6][K/32]; bit k
 * % 32 of word k / 32 of row key: every ordered key, each expanded from the
 * device's row of its unordered cell pair), synchronous. SC_ERR_INVALID_ARG
 * if the scene was built without one; SC_ERR_OOM if the host staging buffer
 * cannot be allocated. */
sc_status sc_scene_export_bit_table(const sc_scene* scene, uint32_t* out);

/*
 * Trace `n` rays (device float32 [n][8]: ox oy oz tmin dx dy dz tmax) with
 * Alg. 4 (d_rays and d_hits 16-byte aligned, d_extra 8-byte aligned):
 * stack traversal, nearer child first, mask test after every slab
 * hit when SC_TRACE_CULL is set and the scene has masks, leaf triangles by
 * the Moller-Trumbore test; closest hit in [tmin, tmax], equal t resolved to
 * the lower triangle index.
 *  d_hits   device sc_hit[n] (written)
 *  d_extra  device uint32 [n][2] = mask tests, mask culls per ray, or NULL
 *  d_slot_fp device uint32 [2*n_inner], or NULL; with SC_TRACE_SHADOW the
 *           per-slot count of slab hits whose mask test fails is added
 * A ray with a non-finite origin or direction, a zero direction, a NaN tmax
 * or tmin > tmax misses with zero counts. Asynchronous on `stream`. Each
 * call takes one of 1024 per-context queue counters in turn, so at most 1024
 * traces of one context may run at the same time (on different streams).
 */
sc_status sc_trace(const sc_scene* scene, const float* d_rays, uint32_t n, uint32_t flags,
                   sc_hit* d_hits, uint32_t* d_extra, uint32_t* d_slot_fp, void* stream);

/* sc_trace without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation). Arguments, results and errors as sc_trace. The ray-queue
 * counters and, when the trace sorts its rays (SC_TRACE_SORT or the context's
 * launch shape), the sort workspace live in a fixed device array of this
 * library, one per GPU (about 65 MiB, held until the process ends), instead
 * of the context's counters and allocator: a sorted trace takes at most
 * 4,194,304 rays (SC_ERR_INVALID_ARG beyond, before any HIP call); an
 * unsorted one any count sc_trace takes. Every call on a GPU shares that
 * GPU's array and leaves its contents behind (each launch clears its counters
 * itself), so calls that overlap on one GPU -- on different streams, or from
 * different contexts or threads -- race and must not be issued; serialise
 * them on one stream. */
sc_status sc_trace_noalloc(const sc_scene* scene, const float* d_rays, uint32_t n, uint32_t flags,
                           sc_hit* d_hits, uint32_t* d_extra, uint32_t* d_slot_fp, void* stream);

/* The order in which a sorted trace takes the rays: d_order (device uint32
 * [n], 4-byte aligned, written) lists ray indices by ascending Morton code
 * of the ray origin, quantised to 256 cells per axis of the scene's vertex
 * bounds (origins outside are clamped, NaN goes to cell 0); equal codes keep
 * index order. A scheduling aid for coherent traversal (not in the paper):
 * it changes no result. Asynchronous on `stream`; the workspace (16 bytes
 * per ray plus counts) comes from the context allocator. */
sc_status sc_ray_order(const sc_scene* scene, const float* d_rays, uint32_t n, uint32_t* d_order,
                       void* stream);

/* Select the traversal launch shape for later sc_trace / sc_trace_batch /
 * sc_batch_create calls on this context (default 256, 8, 1, 8, 0, 0, 0, 16,
 * 16). Errors: SC_ERR_INVALID_ARG (NULL pointer, a field out of its range),
 * SC_ERR_UNSUPPORTED (an uncompiled (block, stack) pair); the context keeps
 * its previous shape on error. sc_get_tune copies the current shape. The
 * shape is read when a trace is issued: traces already queued keep theirs. */
sc_status sc_set_tune(sc_ctx* ctx, const sc_tune* tune);
sc_status sc_get_tune(const sc_ctx* ctx, sc_tune* out);

/* Device checks, a debugging aid for callers (not part of the method).
 * With on != 0, later sc_trace / sc_trace_noalloc / sc_trace_batch calls and
 * batches created afterwards (a batch keeps the kernels it was recorded with)
 * run kernels that compare every inner-node reference with the scene's node
 * count, every leaf's triangle range with its triangle count, every stack push
 * with the lane's stack capacity and every tested codebook index with K before
 * using it. A failed check does not read or write out of range: it ORs its bit
 * into the context's check word (SC_CHECK_NODE, SC_CHECK_TRI, SC_CHECK_STACK,
 * SC_CHECK_INDEX), and the ray ends with the hit it has, or the stack entry is
 * dropped; results then differ from an unchecked trace. Passing checks change
 * no result. Enabling allocates the 4-byte check word once (synchronous,
 * zeroed). Errors: SC_ERR_INVALID_ARG (ctx NULL), SC_ERR_OOM. */
#define SC_CHECK_NODE 1u
#define SC_CHECK_TRI 2u
#define SC_CHECK_STACK 4u
#define SC_CHECK_INDEX 8u
sc_status sc_set_device_checks(sc_ctx* ctx, int on);
/* The bits the failed checks set since the last reset (0 before checks were
 * ever enabled); synchronises the device; reset != 0 clears the word.
 * Errors: SC_ERR_INVALID_ARG (NULL pointer), SC_ERR_HIP. */
sc_status sc_get_check_flags(sc_ctx* ctx, uint32_t* out, int reset);
/* Lower the checked limits below the scene's own (0 keeps a limit at the
 * scene's value): at most max_stack stack entries a lane, inner-node
 * references below max_nodes, triangle ranges ending at or below max_tris.
 * The buffers stay as large as they are, so a lowered limit makes a check
 * fail without any access out of range -- how the checks themselves are
 * tested. Read when a trace is issued. Errors: SC_ERR_INVALID_ARG. */
sc_status sc_set_check_limits(sc_ctx* ctx, uint32_t max_stack, uint32_t max_nodes, uint32_t max_tris);

/* One scene's rays in a batched launch. All items of a batch must come from
 * one context and share the mask mode, R, the node width (2 or 4) and, for
 * 4-wide scenes, the child-box storage (float or quantised). d_rays/d_hits as
 * in sc_trace; d_extra and d_slot_fp may be NULL. Compressed masks are read
 * from each scene's codebook (no LDS copy, no bit table). */
typedef struct {
    const sc_scene* scene;
    const float* d_rays;
    uint32_t n;
    sc_hit* d_hits;
    uint32_t* d_extra;
    uint32_t* d_slot_fp;
} sc_batch_item;

typedef struct sc_batch sc_batch;

/* Trace several scenes' rays in one persistent launch: the items form one
 * ray queue (largest estimated work first), every lane takes its next ray
 * from any item, so uneven scene sizes keep the GPU busy. Results equal
 * sc_trace on each item alone. flags: SC_TRACE_CULL, SC_TRACE_SHADOW and
 * SC_TRACE_SORT; with SC_TRACE_SORT (or the launch shape's sort) the rays are
 * taken in the order of (item, Morton code of the origin in that item's
 * scene bounds), which keeps the items' order (at most 256 items, else
 * SC_ERR_UNSUPPORTED; workspace of 16 bytes per ray plus counts from the
 * context allocator, or held by the batch for sc_batch_create).
 * The launch shape is the context's (sc_set_tune); a replayable graph of the
 * same launch comes from sc_batch_create. Synchronises `stream` (the
 * descriptor table uploaded for the call is released afterwards);
 * sc_batch_launch does not. */
sc_status sc_trace_batch(sc_ctx* ctx, const sc_batch_item* items, uint32_t n_items, uint32_t flags,
                         void* stream);

/* The same launch recorded once into a HIP graph (counter reset kernel +
 * traversal kernel, with the context's current launch shape; a sorted batch
 * also records the ordering kernels, so every replay orders the rays' current
 * contents) for cheap replays: sc_batch_launch replays it on `stream`. The item buffers are
 * bound at creation; their contents may change between replays. Replays of
 * one batch share its queue counters: keep them on one stream. */
sc_status sc_batch_create(sc_ctx* ctx, const sc_batch_item* items, uint32_t n_items, uint32_t flags,
                          sc_batch** out);
sc_status sc_batch_launch(sc_batch* batch, void* stream);
sc_status sc_batch_destroy(sc_batch* batch); /* NULL-safe */

/* The ray-mask LUT of resolution R as built on the device (Sect. 3.1.1):
 * d_out receives R^6 entries of words(R) uint64 (words = 1 for R=4, 4 for
 * R=6); entry key ((((bx*R+by)*R+bz)*R+ex)*R+ey)*R+ez, voxel bit x+R*y+R^2*z. */
sc_status sc_raymask_lut(sc_ctx* ctx, uint32_t R, uint64_t* d_out, void* stream);

/* Alg. 3 on the device for arbitrary masks and codebook (checks and tools):
 * d_masks [n][words], d_codebook [K][words] sorted by set-bit count, output
 * d_idx [n] uint16 = index of the tightest superset. K multiple of 64, <= 4096. */
sc_status sc_compress_masks(sc_ctx* ctx, uint32_t R, const uint64_t* d_codebook, uint32_t K,
                            const uint64_t* d_masks, uint32_t n, uint16_t* d_idx, void* stream);

/* ---------------------------------------------------------------------------
 * Learned mask placement. A small MLP predicts, from a child slot's geometry,
 * how many false-positive box hits its mask would remove; masks go to the
 * slots with the highest predictions under a memory budget (SC_MASK_SPARSE).
 * Skipping a mask is always conservative, so any placement keeps the exact
 * hits of the method with all masks.
 * ------------------------------------------------------------------------ */
#define SC_MLP_PARAMS 5057 /* W1[64][12] b1[64] W2[64][64] b2[64] W3[64] b3 */

/* 12 float features per child slot (d_out [2*n_inner][12], device), for a
 * scene built with masks (RAW, LUT or SPARSE): extents relative to the parent
 * box (x, y, z), log2(area / root area) / 32, parent depth / tree depth,
 * log2(1 + triangles) / 24, occupied fraction of its exact mask, the mean
 * over its triangles of thinness (1 - 4 sqrt(3) area / sum of squared
 * edges), the centre of its box relative to the root box (x, y, z: 0 at the
 * root's low face, 1 at its high face; 0 on an axis where the root is flat),
 * then 1 if the child is a leaf. Synchronises `stream`. */
sc_status sc_slot_features(const sc_scene* scene, float* d_out, void* stream);

/* y[n] = MLP(x[n][12]); d_act [n][128] receives both pre-activation layers
 * for the backward pass, or may be NULL. */
sc_status sc_mlp_forward(sc_ctx* ctx, const float* d_params, const float* d_x, uint32_t n, float* d_y,
                         float* d_act, void* stream);

/* Gradient of the mean squared error (1/n) sum (y - t)^2 with respect to the
 * parameters (d_grad [SC_MLP_PARAMS]), from the forward pass's d_y and d_act.
 * d_work: device scratch of SC_MLP_WORK_FLOATS(n) floats. d_loss (one float)
 * or NULL. Batch sums run in a fixed order (SC_MLP_GRAD_PARTS contiguous
 * sample ranges, each summed in index order, then the ranges in order), so the
 * result is deterministic. */
#define SC_MLP_GRAD_PARTS 32
#define SC_MLP_WORK_FLOATS(n) ((size_t)(n) * 130 + (size_t)SC_MLP_GRAD_PARTS * SC_MLP_PARAMS)
sc_status sc_mlp_backward(sc_ctx* ctx, const float* d_params, const float* d_x, const float* d_act,
                          const float* d_y, const float* d_t, uint32_t n, float* d_grad, float* d_work,
                          float* d_loss, void* stream);

/* One Adam step (Kingma & Ba 2015) on all parameters; step counts from 1. */
sc_status sc_mlp_adam(sc_ctx* ctx, float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t step,
                      float lr, float beta1, float beta2, float eps, void* stream);

/* Host: mark the n_place slots with the highest scores (ties: lower slot
 * first; a NaN score counts as -infinity) in h_placement [n_slots]
 * (1 = carries a mask). */
sc_status sc_place_top(const float* h_scores, uint32_t n_slots, uint32_t n_place, uint8_t* h_placement);

const char* sc_status_string(sc_status s);
const char* sc_last_error(void);  /* thread-local detail of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* SUBCULL_H */
