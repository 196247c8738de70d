/*
 * CPU ORACLE for subspace culling (Yoshimura & Harada, "Subspace Culling for
 * Ray-Box Intersection", 2023).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
 * HIP path is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code, header,
 * table or constant generator with the HIP library, and the product path
 * never calls it.
 *
 * Precision: every decision that ends in an integer (hit id, test counts,
 * mask bits, codebook index) is taken in float32 with the exact expression
 * order of the traversal kernels, because the method's outputs are integers
 * decided by float32 geometry. Surface-area costs and importances are
 * float64. Build with -O2 -ffp-contract=off (no fused multiply-add, no fast
 * math) so that every float32 operation rounds exactly once.
 *
 * min2/max2 below are the ternaries (a<b)?a:b and (a>b)?a:b: a NaN operand
 * in the second position is ignored, and the fold order fixes the sign of
 * zero, so both sides agree to the bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_OOM 3
#define ORC_ERR_DEPTH 4

#define LEAF_BIT 0x80000000u
#define EMPTY_REF 0xFFFFFFFFu
#define NO_HIT 0xFFFFFFFFu

static inline float min2f(float a, float b) { return (a < b) ? a : b; }
static inline float max2f(float a, float b) { return (a > b) ? a : b; }
static inline float min3f(float a, float b, float c) { return min2f(min2f(a, b), c); }
static inline float max3f(float a, float b, float c) { return max2f(max2f(a, b), c); }

static inline uint32_t words_for(uint32_t R) { return (R * R * R + 63u) / 64u; }
static uint32_t popc(const uint64_t* m, uint32_t W);

/* ------------------------------------------------------------------------
 * 1. BVH construction: binned SAH (Sect. 4 names a binned SAH builder; the
 *    split cost is the SAH of Eq. 1 with a size-based leaf rule, so the two
 *    cost constants of Eq. 1 drop out of the split choice).
 *    - triangle box = componentwise min/max of its three vertices
 *    - centroid = (lo + hi) * 0.5f
 *    - node box over a range = fold of triangle boxes in current order
 *    - leaf iff count <= leaf_max
 *    - per axis with a non-empty centroid extent: bin = floor((c - lo) *
 *      (bins / extent)) clamped to bins-1; cost(s) = SA(L)*nL + SA(R)*nR in
 *      float64; first strict minimum over (axis asc, s asc) wins
 *    - no valid split: split at the middle of the current order
 *    - stable partition; left subtree first; inner nodes numbered in DFS
 *      pre-order; triangles end up in leaf order.
 * ---------------------------------------------------------------------- */
typedef struct { float lo[3], hi[3]; } Box;

typedef struct {
    const float* tris;
    uint32_t n, leaf_max, bins, depth_cap;
    uint32_t* idx;
    uint32_t* tmp;
    Box* tbox;
    float* cent;      /* [n][3] */
    float* cbox;      /* [n_inner][12] */
    uint32_t* cref;   /* [n_inner][2] */
    uint32_t* range;  /* [n_inner][2] first, count */
    uint32_t n_inner, depth;
    int err;
} Builder;

static void box_empty(Box* b) {
    for (int j = 0; j < 3; ++j) { b->lo[j] = INFINITY; b->hi[j] = -INFINITY; }
}

static void box_grow(Box* b, const Box* x) {
    for (int j = 0; j < 3; ++j) {
        b->lo[j] = (x->lo[j] < b->lo[j]) ? x->lo[j] : b->lo[j];
        b->hi[j] = (x->hi[j] > b->hi[j]) ? x->hi[j] : b->hi[j];
    }
}

static double box_area(const Box* b) {
    double dx = (double)b->hi[0] - (double)b->lo[0];
    double dy = (double)b->hi[1] - (double)b->lo[1];
    double dz = (double)b->hi[2] - (double)b->lo[2];
    return 2.0 * ((dx * dy + dy * dz) + dz * dx);
}

static inline uint32_t bin_of(float c, float lo, float scale, uint32_t bins) {
    float f = (c - lo) * scale;
    if (f >= (float)(bins - 1)) return bins - 1;
    return (uint32_t)(int)f;
}

static uint32_t build_rec(Builder* B, uint32_t b, uint32_t e, uint32_t level, Box* out) {
    Box box;
    box_empty(&box);
    for (uint32_t i = b; i < e; ++i) box_grow(&box, &B->tbox[B->idx[i]]);
    *out = box;
    uint32_t count = e - b;
    if (count <= B->leaf_max) return LEAF_BIT | b | ((count - 1u) << 29);
    if (level > B->depth_cap) { B->err = ORC_ERR_DEPTH; return 0; }
    if (level > B->depth) B->depth = level;
    uint32_t node = B->n_inner++;
    B->range[2 * node + 0] = b;
    B->range[2 * node + 1] = count;

    Box cb;
    box_empty(&cb);
    for (uint32_t i = b; i < e; ++i) {
        const float* c = &B->cent[3 * (size_t)B->idx[i]];
        for (int j = 0; j < 3; ++j) {
            cb.lo[j] = (c[j] < cb.lo[j]) ? c[j] : cb.lo[j];
            cb.hi[j] = (c[j] > cb.hi[j]) ? c[j] : cb.hi[j];
        }
    }
    double best_cost = INFINITY;
    int best_axis = -1;
    uint32_t best_s = 0;
    float best_scale = 0.0f;
    uint32_t nb = B->bins;
    uint32_t cnt[256];
    Box bb[256], pre[256];
    for (int a = 0; a < 3; ++a) {
        if (!(cb.hi[a] > cb.lo[a])) continue;
        float scale = (float)nb / (cb.hi[a] - cb.lo[a]);
        if (!isfinite(scale)) continue;
        for (uint32_t k = 0; k < nb; ++k) { cnt[k] = 0; box_empty(&bb[k]); }
        for (uint32_t i = b; i < e; ++i) {
            uint32_t t = B->idx[i];
            uint32_t k = bin_of(B->cent[3 * (size_t)t + a], cb.lo[a], scale, nb);
            cnt[k]++;
            box_grow(&bb[k], &B->tbox[t]);
        }
        /* pre[s] = union of bins [0, s) for s = 1..nb-1 */
        Box acc;
        box_empty(&acc);
        for (uint32_t s = 1; s < nb; ++s) { box_grow(&acc, &bb[s - 1]); pre[s] = acc; }
        uint32_t nleft[256];
        uint32_t run = 0;
        for (uint32_t s = 1; s < nb; ++s) { run += cnt[s - 1]; nleft[s] = run; }
        /* suffix sweep from the right, evaluating each boundary */
        Box suf;
        box_empty(&suf);
        uint32_t nright = 0;
        double cost_s[256];
        for (uint32_t s = nb - 1; s >= 1; --s) {
            box_grow(&suf, &bb[s]);
            nright += cnt[s];
            uint32_t nl = nleft[s];
            if (nl == 0 || nright == 0) { cost_s[s] = INFINITY; continue; }
            cost_s[s] = box_area(&pre[s]) * (double)nl + box_area(&suf) * (double)nright;
        }
        for (uint32_t s = 1; s < nb; ++s) {
            if (cost_s[s] < best_cost) {
                best_cost = cost_s[s];
                best_axis = a;
                best_s = s;
                best_scale = scale;
            }
        }
    }
    uint32_t mid;
    if (best_axis >= 0) {
        uint32_t w = b;
        for (uint32_t i = b; i < e; ++i) {
            uint32_t t = B->idx[i];
            if (bin_of(B->cent[3 * (size_t)t + best_axis], cb.lo[best_axis], best_scale, nb) < best_s)
                B->tmp[w++] = t;
        }
        mid = w;
        for (uint32_t i = b; i < e; ++i) {
            uint32_t t = B->idx[i];
            if (!(bin_of(B->cent[3 * (size_t)t + best_axis], cb.lo[best_axis], best_scale, nb) < best_s))
                B->tmp[w++] = t;
        }
        memcpy(&B->idx[b], &B->tmp[b], (size_t)count * sizeof(uint32_t));
    } else {
        mid = b + count / 2u;
    }
    Box lb, rb;
    uint32_t l = build_rec(B, b, mid, level + 1, &lb);
    if (B->err) return 0;
    uint32_t r = build_rec(B, mid, e, level + 1, &rb);
    if (B->err) return 0;
    float* cbx = &B->cbox[12 * (size_t)node];
    for (int j = 0; j < 3; ++j) {
        cbx[j] = lb.lo[j]; cbx[3 + j] = lb.hi[j];
        cbx[6 + j] = rb.lo[j]; cbx[9 + j] = rb.hi[j];
    }
    B->cref[2 * node + 0] = l;
    B->cref[2 * node + 1] = r;
    return node;
}

/* info[0] = inner node count, info[1] = root ref, info[2] = depth (inner
 * nodes on the longest root-to-leaf path). Output arrays hold max(n,1)
 * entries. */
int orc_bvh_build(const float* tris, uint32_t n, uint32_t leaf_max, uint32_t bins,
                  uint32_t depth_cap, float* cbox, uint32_t* cref, uint32_t* range,
                  uint32_t* perm, uint32_t* info) {
    if (leaf_max < 1 || leaf_max > 4 || bins < 2 || bins > 256 || n >= (1u << 29)) return ORC_ERR_ARG;
    for (size_t i = 0; i < 9 * (size_t)n; ++i)
        if (!isfinite(tris[i])) return ORC_ERR_ARG;
    info[0] = 0; info[1] = EMPTY_REF; info[2] = 0;
    if (n == 0) return ORC_OK;
    Builder B;
    memset(&B, 0, sizeof B);
    B.tris = tris; B.n = n; B.leaf_max = leaf_max; B.bins = bins; B.depth_cap = depth_cap;
    B.idx = perm;
    B.tmp = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    B.tbox = (Box*)malloc((size_t)n * sizeof(Box));
    B.cent = (float*)malloc((size_t)n * 3 * sizeof(float));
    if (!B.tmp || !B.tbox || !B.cent) { free(B.tmp); free(B.tbox); free(B.cent); return ORC_ERR_OOM; }
    B.cbox = cbox; B.cref = cref; B.range = range;
    for (uint32_t t = 0; t < n; ++t) {
        const float* v = &tris[9 * (size_t)t];
        for (int j = 0; j < 3; ++j) {
            float lo = min2f(min2f(v[j], v[3 + j]), v[6 + j]);
            float hi = max2f(max2f(v[j], v[3 + j]), v[6 + j]);
            B.tbox[t].lo[j] = lo;
            B.tbox[t].hi[j] = hi;
            B.cent[3 * (size_t)t + j] = (lo + hi) * 0.5f;
        }
        perm[t] = t;
    }
    Box root;
    uint32_t rr = build_rec(&B, 0, n, 1, &root);
    free(B.tmp); free(B.tbox); free(B.cent);
    if (B.err) return B.err;
    info[0] = B.n_inner; info[1] = rr; info[2] = B.depth;
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * 2. Ray-mask LUT (Sect. 3.1.1 and Alg. 1): entry (beg, end) is the set of
 *    voxels that a unit cell swept from cell beg to cell end overlaps, i.e.
 *    voxel v is set iff some s in [0,1] has |beg_i + s*(end_i-beg_i) - v_i|
 *    < 1 on all three axes (the AABB-AABB sweep, with strict overlap). With
 *    the time scaled by 60 every interval end is an integer for R <= 6.
 *    Key = ((((bx*R+by)*R+bz)*R+ex)*R+ey)*R+ez; voxel bit = x + R*y + R^2*z.
 * ---------------------------------------------------------------------- */
int orc_raymask_lut(uint32_t R, uint64_t* out) {
    if (R < 1 || R > 6) return ORC_ERR_ARG;
    const int T = 60;
    uint32_t W = words_for(R);
    uint32_t R3 = R * R * R;
    for (uint32_t kb = 0; kb < R3; ++kb) {
        int beg[3] = {(int)(kb / (R * R)), (int)((kb / R) % R), (int)(kb % R)};
        for (uint32_t ke = 0; ke < R3; ++ke) {
            int end[3] = {(int)(ke / (R * R)), (int)((ke / R) % R), (int)(ke % R)};
            uint64_t* m = &out[((size_t)kb * R3 + ke) * W];
            for (uint32_t w = 0; w < W; ++w) m[w] = 0;
            for (uint32_t z = 0; z < R; ++z)
                for (uint32_t y = 0; y < R; ++y)
                    for (uint32_t x = 0; x < R; ++x) {
                        int v[3] = {(int)x, (int)y, (int)z};
                        int lo = -1000000, hi = 1000000, ok = 1;
                        for (int i = 0; i < 3; ++i) {
                            int d = end[i] - beg[i];
                            if (d == 0) {
                                if (v[i] != beg[i]) ok = 0;
                                continue;
                            }
                            int a = T * (v[i] - 1 - beg[i]) / d;
                            int b = T * (v[i] + 1 - beg[i]) / d;
                            if (a > b) { int t = a; a = b; b = t; }
                            if (a > lo) lo = a;
                            if (b < hi) hi = b;
                        }
                        if (ok && lo < hi && lo < T && hi > 0) {
                            uint32_t bit = x + R * y + R * R * z;
                            m[bit >> 6] |= 1ull << (bit & 63);
                        }
                    }
        }
    }
    return ORC_OK;
}

/* Ray-mask table at ray resolution 2R (Sect. 4.2 compares R_ray = R and
 * R_ray = 2R): the key holds the entry and exit cells on the twice finer grid
 * F = 2R, ((((bx*F+by)*F+bz)*F+ex)*F+ey)*F+ez; the value is the R-grid mask
 * of the coarse voxels that contain a fine voxel of the strict sweep between
 * the two fine cells (the definition of the R table applied at F, each fine
 * voxel v then mapped to coarse voxel v / 2). Exact integer arithmetic with
 * the sweep parameter scaled by 27720 (divisible by every |e - b| <= 11). */
int orc_raymask_lut2(uint32_t R, uint64_t* out) {
    if (R < 1 || R > 6) return ORC_ERR_ARG;
    const int64_t T = 27720;
    const int F = 2 * (int)R;
    uint32_t W = words_for(R);
    size_t keys = (size_t)F * F * F * F * F * F;
    for (size_t key = 0; key < keys; ++key) {
        size_t q = key;
        int e[3], b[3];
        e[2] = (int)(q % F); q /= F;
        e[1] = (int)(q % F); q /= F;
        e[0] = (int)(q % F); q /= F;
        b[2] = (int)(q % F); q /= F;
        b[1] = (int)(q % F); q /= F;
        b[0] = (int)q;
        uint64_t* m = &out[key * W];
        for (uint32_t w = 0; w < W; ++w) m[w] = 0;
        int vlo[3], vhi[3];
        for (int i = 0; i < 3; ++i) {
            vlo[i] = b[i] < e[i] ? b[i] : e[i];
            vhi[i] = b[i] < e[i] ? e[i] : b[i];
        }
        for (int z = vlo[2]; z <= vhi[2]; ++z)
            for (int y = vlo[1]; y <= vhi[1]; ++y)
                for (int x = vlo[0]; x <= vhi[0]; ++x) {
                    int v[3] = {x, y, z};
                    int64_t lo = -((int64_t)1 << 40), hi = (int64_t)1 << 40;
                    int ok = 1;
                    for (int i = 0; i < 3; ++i) {
                        int64_t d = e[i] - b[i];
                        if (d == 0) {
                            if (v[i] != b[i]) ok = 0;
                            continue;
                        }
                        int64_t a = T * (v[i] - 1 - b[i]) / d;
                        int64_t c = T * (v[i] + 1 - b[i]) / d;
                        if (a > c) { int64_t t = a; a = c; c = t; }
                        if (a > lo) lo = a;
                        if (c < hi) hi = c;
                    }
                    if (ok && lo < hi && lo < T && hi > 0) {
                        uint32_t bit = (uint32_t)(x / 2) + R * (uint32_t)(y / 2) + R * R * (uint32_t)(z / 2);
                        m[bit >> 6] |= 1ull << (bit & 63);
                    }
                }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * 3. Object masks with L = infinity (Sect. 3.1.1, 3.2.1): bit v of a node is
 *    set iff some triangle of the node's subtree overlaps voxel v of the
 *    node box, each voxel dilated by delta so that float32 rounding in the
 *    ray-side computation stays inside the mask. Overlap is the separating
 *    axis test (3 box normals, 9 edge-by-axis cross products, the triangle
 *    normal): separated iff on some axis the three projected vertices all
 *    lie above +r or below -r, r being the projected half-size of the box.
 *    voxel k on axis j: centre lo + (k + 0.5f) * w, half-size 0.5f * w +
 *    delta, w = (hi - lo) / R.
 * ---------------------------------------------------------------------- */
static int tri_box_overlap(const float* v, const float c[3], const float h[3]) {
    float a[3], b[3], q[3];
    for (int j = 0; j < 3; ++j) {
        a[j] = v[j] - c[j];
        b[j] = v[3 + j] - c[j];
        q[j] = v[6 + j] - c[j];
    }
    /* box normals */
    for (int j = 0; j < 3; ++j)
        if (min3f(a[j], b[j], q[j]) > h[j] || max3f(a[j], b[j], q[j]) < -h[j]) return 0;
    float f[3][3];
    for (int j = 0; j < 3; ++j) {
        f[0][j] = b[j] - a[j];
        f[1][j] = q[j] - b[j];
        f[2][j] = a[j] - q[j];
    }
    const float* P[3] = {a, b, q};
    for (int k = 0; k < 3; ++k) {
        const float* e = f[k];
        float p[3], r;
        /* x-axis cross edge: axis (0, -e.z, e.y) */
        for (int i = 0; i < 3; ++i) p[i] = e[1] * P[i][2] - e[2] * P[i][1];
        r = h[1] * fabsf(e[2]) + h[2] * fabsf(e[1]);
        if (min3f(p[0], p[1], p[2]) > r || max3f(p[0], p[1], p[2]) < -r) return 0;
        /* y-axis cross edge: axis (e.z, 0, -e.x) */
        for (int i = 0; i < 3; ++i) p[i] = e[2] * P[i][0] - e[0] * P[i][2];
        r = h[0] * fabsf(e[2]) + h[2] * fabsf(e[0]);
        if (min3f(p[0], p[1], p[2]) > r || max3f(p[0], p[1], p[2]) < -r) return 0;
        /* z-axis cross edge: axis (-e.y, e.x, 0) */
        for (int i = 0; i < 3; ++i) p[i] = e[0] * P[i][1] - e[1] * P[i][0];
        r = h[0] * fabsf(e[1]) + h[1] * fabsf(e[0]);
        if (min3f(p[0], p[1], p[2]) > r || max3f(p[0], p[1], p[2]) < -r) return 0;
    }
    /* triangle normal n = f0 x f1 */
    float nx = f[0][1] * f[1][2] - f[0][2] * f[1][1];
    float ny = f[0][2] * f[1][0] - f[0][0] * f[1][2];
    float nz = f[0][0] * f[1][1] - f[0][1] * f[1][0];
    float p[3];
    for (int i = 0; i < 3; ++i) p[i] = (nx * P[i][0] + ny * P[i][1]) + nz * P[i][2];
    float r = (h[0] * fabsf(nx) + h[1] * fabsf(ny)) + h[2] * fabsf(nz);
    if (min3f(p[0], p[1], p[2]) > r || max3f(p[0], p[1], p[2]) < -r) return 0;
    return 1;
}

/* OR the voxels of box (lo, hi) that triangle v overlaps into m. The
 * per-axis pre-check is the box-normal part of the same test, evaluated
 * with the same values, so skipping voxels that fail it changes nothing. */
static void voxelize_tri(const float* v, const float* lo, const float* hi, uint32_t R,
                         float delta, uint64_t* m) {
    float w[3], h[3];
    int pass[3][8];
    for (int j = 0; j < 3; ++j) {
        w[j] = (hi[j] - lo[j]) / (float)R;
        h[j] = 0.5f * w[j] + delta;
        for (uint32_t k = 0; k < R; ++k) {
            float c = lo[j] + ((float)k + 0.5f) * w[j];
            float a = v[j] - c, b = v[3 + j] - c, q = v[6 + j] - c;
            pass[j][k] = !(min3f(a, b, q) > h[j] || max3f(a, b, q) < -h[j]);
        }
    }
    for (uint32_t z = 0; z < R; ++z) {
        if (!pass[2][z]) continue;
        for (uint32_t y = 0; y < R; ++y) {
            if (!pass[1][y]) continue;
            for (uint32_t x = 0; x < R; ++x) {
                if (!pass[0][x]) continue;
                float c[3] = {lo[0] + ((float)x + 0.5f) * w[0], lo[1] + ((float)y + 0.5f) * w[1],
                              lo[2] + ((float)z + 0.5f) * w[2]};
                if (tri_box_overlap(v, c, h)) {
                    uint32_t bit = x + R * y + R * R * z;
                    m[bit >> 6] |= 1ull << (bit & 63);
                }
            }
        }
    }
}

static void slot_range(const uint32_t* cref, const uint32_t* range, uint32_t slot,
                       uint32_t* first, uint32_t* count) {
    uint32_t ref = cref[slot];
    if (ref & LEAF_BIT) { *first = ref & 0x1FFFFFFFu; *count = ((ref >> 29) & 3u) + 1u; }
    else { *first = range[2 * ref]; *count = range[2 * ref + 1]; }
}

/* One mask per child slot (node i, child c) -> out[(2*i+c)*W .. +W). */
int orc_object_masks(const float* tris, const uint32_t* perm, uint32_t n_inner, const float* cbox,
                     const uint32_t* cref, const uint32_t* range, uint32_t R, float delta,
                     uint64_t* out, int nthreads) {
    if (R < 1 || R > 6) return ORC_ERR_ARG;
    uint32_t W = words_for(R);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t s = 0; s < 2 * (int64_t)n_inner; ++s) {
        uint64_t* m = &out[(size_t)s * W];
        for (uint32_t w = 0; w < W; ++w) m[w] = 0;
        const float* bx = &cbox[12 * (size_t)(s >> 1) + 6 * (size_t)(s & 1)];
        uint32_t first, count;
        slot_range(cref, range, (uint32_t)s, &first, &count);
        for (uint32_t j = first; j < first + count; ++j)
            voxelize_tri(&tris[9 * (size_t)perm[j]], bx, bx + 3, R, delta, m);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * 3b. Approximate object masks (Sect. 3.2.1, Alg. 2). The mask of child
 *     slot s (node N, box P) takes the occupancy from N's subtree down to L
 *     levels: the triangles of every leaf within L levels are voxelized
 *     exactly into P's grid (as in 3.), and every inner node exactly L
 *     levels down contributes its own approximate mask through Alg. 2: each
 *     set voxel of that child box C fills the box-shaped block of P's
 *     voxels its extent projects to, read from the filling-pattern table.
 *     Leaf slots are always exact; L >= the subtree height gives the exact
 *     mask.
 *     Projection (float64): for child grid border i = 0..R,
 *       b_i = cLo + (i * cExt) / R,
 *       lo index = floor((R * ((b_i - 2 delta) - pLo)) / pExt),
 *       hi index = floor((R * ((b_i + 2 delta) - pLo)) / pExt),
 *     clamped to [0, R-1]; child voxel x fills parent indices
 *     [lo index of border x, hi index of border x+1]. A parent axis of zero
 *     extent is filled whole (as the exact mask sets every voxel of it).
 *     The 2 delta margin keeps the result a superset of the exact mask under
 *     rounding.
 *     Filling-pattern table key ((((x0*R+y0)*R+z0)*R+x1)*R+y1)*R+z1: the
 *     voxels with x0<=x<=x1, y0<=y<=y1, z0<=z<=z1.
 * ---------------------------------------------------------------------- */
int orc_fill_table(uint32_t R, uint64_t* out) {
    if (R < 1 || R > 6) return ORC_ERR_ARG;
    uint32_t W = words_for(R);
    size_t keys = (size_t)R * R * R * R * R * R;
    for (size_t k = 0; k < keys; ++k) {
        size_t q = k;
        uint32_t z1 = q % R; q /= R;
        uint32_t y1 = q % R; q /= R;
        uint32_t x1 = q % R; q /= R;
        uint32_t z0 = q % R; q /= R;
        uint32_t y0 = q % R; q /= R;
        uint32_t x0 = (uint32_t)q;
        uint64_t* m = &out[k * W];
        for (uint32_t w = 0; w < W; ++w) m[w] = 0;
        for (uint32_t z = z0; z <= z1; ++z)
            for (uint32_t y = y0; y <= y1; ++y)
                for (uint32_t x = x0; x <= x1; ++x) {
                    uint32_t bit = x + R * y + R * R * z;
                    m[bit >> 6] |= 1ull << (bit & 63);
                }
    }
    return ORC_OK;
}

static int clamp_index(double u, uint32_t R) {
    double f = floor(u);
    if (!(f > 0.0)) return 0;
    if (f > (double)(R - 1)) return (int)(R - 1);
    return (int)f;
}

/* Alg. 2: OR into m (box P = plo..phi) the filling patterns of the set
 * voxels of child mask cm (box C = clo..chi). */
static void fill_from_child(uint64_t* m, const float* plo, const float* phi, const uint64_t* cm, const float* clo,
                           const float* chi, uint32_t R, float delta, const uint64_t* table) {
    uint32_t W = words_for(R);
    int lo_idx[3][7], hi_idx[3][7];
    for (int j = 0; j < 3; ++j) {
        double pl = (double)plo[j], pe = (double)phi[j] - (double)plo[j];
        double cl = (double)clo[j], ce = (double)chi[j] - (double)clo[j];
        for (uint32_t i = 0; i <= R; ++i) {
            if (!(pe > 0.0)) {
                lo_idx[j][i] = 0;
                hi_idx[j][i] = (int)R - 1;
                continue;
            }
            double b = cl + ((double)i * ce) / (double)R;
            lo_idx[j][i] = clamp_index(((double)R * ((b - 2.0 * (double)delta) - pl)) / pe, R);
            hi_idx[j][i] = clamp_index(((double)R * ((b + 2.0 * (double)delta) - pl)) / pe, R);
        }
    }
    for (uint32_t z = 0; z < R; ++z)
        for (uint32_t y = 0; y < R; ++y)
            for (uint32_t x = 0; x < R; ++x) {
                uint32_t bit = x + R * y + R * R * z;
                if (!((cm[bit >> 6] >> (bit & 63)) & 1u)) continue;
                size_t key = (((((size_t)lo_idx[0][x] * R + lo_idx[1][y]) * R + lo_idx[2][z]) * R +
                               hi_idx[0][x + 1]) * R + hi_idx[1][y + 1]) * R + hi_idx[2][z + 1];
                const uint64_t* pat = &table[key * W];
                for (uint32_t w = 0; w < W; ++w) m[w] |= pat[w];
            }
}

/* Alg. 2 for one child mask alone (for tests): out = fill of cm into P. */
int orc_fill_one(const float* plo, const float* phi, const uint64_t* cm, const float* clo, const float* chi,
                 uint32_t R, float delta, const uint64_t* table, uint64_t* out) {
    if (R < 1 || R > 6) return ORC_ERR_ARG;
    for (uint32_t w = 0; w < words_for(R); ++w) out[w] = 0;
    fill_from_child(out, plo, phi, cm, clo, chi, R, delta, table);
    return ORC_OK;
}

/* Masks of every child slot with approximation level L (>= 1), computed
 * from the deepest nodes up (nodes are in DFS pre-order, so every
 * descendant has a larger index than its ancestors). */
int orc_approx_masks(const float* tris, const uint32_t* perm, uint32_t n_inner, const float* cbox,
                     const uint32_t* cref, const uint32_t* range, uint32_t R, float delta, uint32_t L,
                     const uint64_t* table, uint64_t* out) {
    if (R < 1 || R > 6 || L < 1 || L > 64) return ORC_ERR_ARG;
    uint32_t W = words_for(R);
    uint32_t st_slot[256], st_lev[256];
    for (int64_t node = (int64_t)n_inner - 1; node >= 0; --node) {
        for (uint32_t c = 0; c < 2; ++c) {
            uint32_t s = 2u * (uint32_t)node + c;
            uint64_t* m = &out[(size_t)s * W];
            for (uint32_t w = 0; w < W; ++w) m[w] = 0;
            const float* P = &cbox[6 * (size_t)s];
            uint32_t r = cref[s];
            if (r & LEAF_BIT) {
                uint32_t first, count;
                slot_range(cref, range, s, &first, &count);
                for (uint32_t j = first; j < first + count; ++j)
                    voxelize_tri(&tris[9 * (size_t)perm[j]], P, P + 3, R, delta, m);
                continue;
            }
            int sp = 0;
            st_slot[sp] = 2u * r + 1u; st_lev[sp] = 1; ++sp;
            st_slot[sp] = 2u * r; st_lev[sp] = 1; ++sp;
            while (sp > 0) {
                --sp;
                uint32_t d = st_slot[sp], k = st_lev[sp];
                uint32_t rd = cref[d];
                if (rd & LEAF_BIT) {
                    uint32_t first, count;
                    slot_range(cref, range, d, &first, &count);
                    for (uint32_t j = first; j < first + count; ++j)
                        voxelize_tri(&tris[9 * (size_t)perm[j]], P, P + 3, R, delta, m);
                } else if (k == L) {
                    const float* Cb = &cbox[6 * (size_t)d];
                    fill_from_child(m, P, P + 3, &out[(size_t)d * W], Cb, Cb + 3, R, delta, table);
                } else {
                    st_slot[sp] = 2u * rd + 1u; st_lev[sp] = k + 1; ++sp;
                    st_slot[sp] = 2u * rd; st_lev[sp] = k + 1; ++sp;
                }
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * 4. Traversal with culling (Alg. 4 with Alg. 1 inside).
 *    slab: per axis x,y,z the near bound n = lo and far bound f = hi when
 *          inv >= 0 (sign bit clear), swapped when inv is negative (PBRT's
 *          form), a = (n-o)*inv, b = (f-o)*inv,
 *          b *= 1 + 3*2^-23 (robust far value), t0 = max2(a, t0),
 *          t1 = min2(b, t1) from t0 = tmin, t1 = best_t; hit iff t0 <= t1.
 *    ray mask (Alg. 1): p = o + t*d at t0 and t1; scale s = R/ext (0 when
 *          ext <= 0 or the quotient is infinite); u = (p - lo)*s clamped to
 *          [0, R-1] (NaN -> 0) and truncated; mask = LUT[beg, end].
 *    order: both children hit -> the one with smaller t0 (tie: child 0)
 *          is visited next, the other is pushed with its t0; a popped entry
 *          whose t0 exceeds best_t is dropped; the root is pushed untested.
 *    leaf: Moller-Trumbore, two-sided, det == 0 rejects; accept t in
 *          [tmin, best_t]; replace iff t < best_t or (t == best_t and the
 *          original id is lower).
 *    counts: box_tests = slab tests, tri_tests = triangle tests, mask_tests
 *          = mask ANDs evaluated, mask_culls = ANDs that were zero.
 *    a child whose stored mask has every bit set is not tested: its AND can
 *          never be zero, since a ray mask always holds the entry cell. In
 *          the sparse mode only the placed slots carry masks.
 * ---------------------------------------------------------------------- */
#define MODE_NONE 0
#define MODE_RAW 1
#define MODE_LUT 2
#define MODE_SPARSE 3
#define FLAG_CULL 1u
#define FLAG_SHADOW 2u

static inline float dot3(const float* a, const float* b) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}
static inline void cross3(const float* a, const float* b, float* r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

static int ray_valid(const float* r) {
    for (int j = 0; j < 4; ++j) if (!isfinite(r[j])) return 0;
    for (int j = 4; j < 7; ++j) if (!isfinite(r[j])) return 0;
    if (isnan(r[7])) return 0;
    if (!(r[3] <= r[7])) return 0;
    if (r[4] == 0.0f && r[5] == 0.0f && r[6] == 0.0f) return 0;
    return 1;
}

typedef struct {
    const float* tris; const uint32_t* perm; const float* cbox; const uint32_t* cref;
    uint32_t root, R, W, mode, flags;
    const uint64_t* masks; const uint64_t* cb; const uint16_t* cidx; const uint64_t* lut;
    const uint8_t* placed;
    float origin_bound;
    uint32_t* slot_fp;
    uint32_t rm_kind;          /* ray mask: 0 table at R, 1 table at 2R (lut2), 2 ideal */
    const uint64_t* lut2;
    uint32_t test_max;         /* the most set bits a tested mask may have (R^3 - 1: all but full) */
    uint32_t* cb_refs;         /* LUT mode, optional: mask tests per codebook entry */
} TraceCtx;

static void raymask_key_cells(const float* lo, const float* hi, const float* o, const float* d,
                              float t, uint32_t R, int cell[3]) {
    for (int j = 0; j < 3; ++j) {
        float ext = hi[j] - lo[j];
        float s = (ext > 0.0f) ? (float)R / ext : 0.0f;
        if (isinf(s)) s = 0.0f;
        float p = o[j] + t * d[j];
        float u = (p - lo[j]) * s;
        u = (u > 0.0f) ? u : 0.0f;
        u = (u < (float)(R - 1)) ? u : (float)(R - 1);
        cell[j] = (int)u;
    }
}

/* "Ideal" ray mask (Sect. 4.1, the grid traversal reference): every voxel of
 * box [lo, hi] whose closed box the segment o + t d, t in [t0, t1], meets,
 * by a float64 slab test per voxel; voxel k on axis j spans
 * [lo + (k ext) / R, lo + ((k + 1) ext) / R]. The triangle side keeps its
 * delta dilation, so the test stays conservative. */
static void ideal_ray_mask(const float* lo, const float* hi, const float* o, const float* d, float t0, float t1,
                           uint32_t R, uint64_t* m) {
    double bl[3][7];
    for (int j = 0; j < 3; ++j) {
        double e = (double)hi[j] - (double)lo[j];
        for (uint32_t k = 0; k <= R; ++k) bl[j][k] = (double)lo[j] + ((double)k * e) / (double)R;
    }
    for (uint32_t z = 0; z < R; ++z)
        for (uint32_t y = 0; y < R; ++y)
            for (uint32_t x = 0; x < R; ++x) {
                uint32_t v[3] = {x, y, z};
                double s0 = (double)t0, s1 = (double)t1;
                int ok = 1;
                for (int j = 0; j < 3 && ok; ++j) {
                    double a = bl[j][v[j]], b = bl[j][v[j] + 1];
                    double oj = (double)o[j], dj = (double)d[j];
                    if (dj == 0.0) {
                        if (oj < a || oj > b) ok = 0;
                        continue;
                    }
                    double ta = (a - oj) / dj, tb = (b - oj) / dj;
                    if (ta > tb) { double t = ta; ta = tb; tb = t; }
                    if (ta > s0) s0 = ta;
                    if (tb < s1) s1 = tb;
                    if (s0 > s1) ok = 0;
                }
                if (ok) {
                    uint32_t bit = x + R * y + R * R * z;
                    m[bit >> 6] |= 1ull << (bit & 63);
                }
            }
}

/* The ideal ray mask alone (for tests). */
int orc_ideal_mask(const float* lo, const float* hi, const float* o, const float* d, float t0, float t1, uint32_t R,
                   uint64_t* out) {
    if (R < 1 || R > 6) return ORC_ERR_ARG;
    for (uint32_t w = 0; w < words_for(R); ++w) out[w] = 0;
    ideal_ray_mask(lo, hi, o, d, t0, t1, R, out);
    return ORC_OK;
}

/* Leaf of Alg. 4: Moller-Trumbore against each triangle of the leaf, in leaf
 * order; the closest t in [tmin, best_t] wins, equal t goes to the lower
 * original triangle id. */
static void leaf_tests(const TraceCtx* C, uint32_t ref, const float* o, const float* d, float tmin,
                       float* best_t, uint32_t* best, uint32_t* tri_tests) {
    uint32_t first = ref & 0x1FFFFFFFu, count = ((ref >> 29) & 3u) + 1u;
    for (uint32_t j = first; j < first + count; ++j) {
        ++*tri_tests;
        uint32_t id = C->perm[j];
        const float* v = &C->tris[9 * (size_t)id];
        float e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
        float e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
        float P[3], Q[3], S[3];
        cross3(d, e2, P);
        float det = dot3(e1, P);
        if (det == 0.0f) continue;
        float idet = 1.0f / det;
        S[0] = o[0] - v[0]; S[1] = o[1] - v[1]; S[2] = o[2] - v[2];
        float u = dot3(S, P) * idet;
        if (u < 0.0f || u > 1.0f) continue;
        cross3(S, e1, Q);
        float vv = dot3(d, Q) * idet;
        if (vv < 0.0f || u + vv > 1.0f) continue;
        float t = dot3(e2, Q) * idet;
        if (t < tmin || t > *best_t) continue;
        if (t < *best_t || (t == *best_t && id < *best)) { *best_t = t; *best = id; }
    }
}

/* Mask test of Sect. 3.1.2 for the child in binary slot `slot` whose box
 * [lo, hi] the ray overlaps over [t0, t1]: the ray mask of the entry and exit
 * cells (Alg. 1) ANDed with the slot's object mask (raw, codebook entry, or
 * absent when not placed). A mask with more than test_max set bits is not
 * tested -- by default only the full mask, which cannot cull; a smaller
 * test_max leaves denser masks untested, which only forgoes culls. Returns 1
 * when the AND is zero (the child can be culled). */
static int mask_test(const TraceCtx* C, uint32_t slot, const float* lo, const float* hi, const float* o,
                     const float* d, float t0, float t1, uint32_t* mask_tests, uint32_t* mask_culls) {
    const uint64_t* om = NULL;
    if (C->mode == MODE_RAW) om = &C->masks[(size_t)slot * C->W];
    else if (C->mode == MODE_LUT) om = &C->cb[(size_t)C->cidx[slot] * C->W];
    else if (C->placed[slot]) om = &C->masks[(size_t)slot * C->W];
    if (!om || popc(om, C->W) > C->test_max) return 0;
    ++*mask_tests;
    if (C->cb_refs && C->mode == MODE_LUT) {
#ifdef _OPENMP
#pragma omp atomic
#endif
        C->cb_refs[C->cidx[slot]] += 1u;
    }
    uint32_t R = C->R;
    uint64_t ideal[4] = {0, 0, 0, 0};
    const uint64_t* rm;
    if (C->rm_kind == 2) {
        ideal_ray_mask(lo, hi, o, d, t0, t1, R, ideal);
        rm = ideal;
    } else {
        uint32_t Q = (C->rm_kind == 1) ? 2 * R : R;
        int cb_[3], ce_[3];
        raymask_key_cells(lo, hi, o, d, t0, Q, cb_);
        raymask_key_cells(lo, hi, o, d, t1, Q, ce_);
        size_t key = (((((size_t)cb_[0] * Q + cb_[1]) * Q + cb_[2]) * Q + ce_[0]) * Q + ce_[1]) * Q + ce_[2];
        rm = (C->rm_kind == 1) ? &C->lut2[key * C->W] : &C->lut[key * C->W];
    }
    uint64_t any = 0;
    for (uint32_t w = 0; w < C->W; ++w) any |= rm[w] & om[w];
    if (any != 0) return 0;
    ++*mask_culls;
    if (C->slot_fp) {
#ifdef _OPENMP
#pragma omp atomic
#endif
        C->slot_fp[slot] += 1u;
    }
    return 1;
}

static void trace_one(const TraceCtx* C, const float* ray, uint32_t* hit, uint32_t* extra) {
    uint32_t box_tests = 0, tri_tests = 0, mask_tests = 0, mask_culls = 0;
    uint32_t best = NO_HIT;
    float best_t = INFINITY;
    if (ray_valid(ray) && C->root != EMPTY_REF) {
        const float o[3] = {ray[0], ray[1], ray[2]};
        const float d[3] = {ray[4], ray[5], ray[6]};
        const float tmin = ray[3];
        float inv[3] = {1.0f / d[0], 1.0f / d[1], 1.0f / d[2]};
        best_t = ray[7];
        int use_mask = (C->mode != MODE_NONE) && (C->flags & (FLAG_CULL | FLAG_SHADOW));
        if (use_mask) {
            float mo = max3f(fabsf(o[0]), fabsf(o[1]), fabsf(o[2]));
            if (mo > C->origin_bound) use_mask = 0;
        }
        int cull = (C->flags & FLAG_CULL) != 0;
        uint32_t st_ref[160];
        float st_t[160];
        int sp = 0;
        st_ref[sp] = C->root; st_t[sp] = tmin; ++sp;
        while (sp > 0) {
            --sp;
            uint32_t ref = st_ref[sp];
            float tn = st_t[sp];
            if (tn > best_t) continue;
            if (ref & LEAF_BIT) {
                leaf_tests(C, ref, o, d, tmin, &best_t, &best, &tri_tests);
                continue;
            }
            const float* nb = &C->cbox[12 * (size_t)ref];
            int hitc[2];
            float t0c[2];
            for (int c = 0; c < 2; ++c) {
                const float* lo = nb + 6 * c;
                const float* hi = lo + 3;
                ++box_tests;
                float t0 = tmin, t1 = best_t;
                for (int j = 0; j < 3; ++j) {
                    /* near bound first: lo for a positive direction, hi for a negative one */
                    int neg = signbit(inv[j]) != 0;
                    float a = ((neg ? hi[j] : lo[j]) - o[j]) * inv[j];
                    float b = ((neg ? lo[j] : hi[j]) - o[j]) * inv[j];
                    b = b * 0x1.000006p0f;
                    t0 = (a > t0) ? a : t0;
                    t1 = (b < t1) ? b : t1;
                }
                hitc[c] = (t0 <= t1);
                t0c[c] = t0;
                if (hitc[c] && use_mask &&
                    mask_test(C, 2u * ref + (uint32_t)c, lo, hi, o, d, t0, t1, &mask_tests, &mask_culls) && cull)
                    hitc[c] = 0;
            }
            const uint32_t* ch = &C->cref[2 * (size_t)ref];
            if (hitc[0] && hitc[1]) {
                int nr = (t0c[1] < t0c[0]) ? 1 : 0;
                int fr = 1 - nr;
                st_ref[sp] = ch[fr]; st_t[sp] = t0c[fr]; ++sp;
                st_ref[sp] = ch[nr]; st_t[sp] = t0c[nr]; ++sp;
            } else if (hitc[0]) {
                st_ref[sp] = ch[0]; st_t[sp] = t0c[0]; ++sp;
            } else if (hitc[1]) {
                st_ref[sp] = ch[1]; st_t[sp] = t0c[1]; ++sp;
            }
        }
    }
    float tout = (best == NO_HIT) ? INFINITY : best_t;
    hit[0] = best;
    memcpy(&hit[1], &tout, 4);
    hit[2] = box_tests;
    hit[3] = tri_tests;
    if (extra) { extra[0] = mask_tests; extra[1] = mask_culls; }
}

int orc_trace_ex(const float* tris, const uint32_t* perm, const float* cbox, const uint32_t* cref,
                 uint32_t root_ref, uint32_t depth, uint32_t R, uint32_t mode, const uint64_t* masks,
                 const uint64_t* codebook, const uint16_t* cidx, const uint8_t* placed, const uint64_t* lut,
                 float origin_bound, uint32_t flags, const float* rays, uint32_t nrays,
                 uint32_t* out_hits, uint32_t* out_extra, uint32_t* slot_fp, int nthreads,
                 uint32_t rm_kind, const uint64_t* lut2, uint32_t test_max);

int orc_trace(const float* tris, const uint32_t* perm, const float* cbox, const uint32_t* cref,
              uint32_t root_ref, uint32_t depth, uint32_t R, uint32_t mode, const uint64_t* masks,
              const uint64_t* codebook, const uint16_t* cidx, const uint8_t* placed, const uint64_t* lut,
              float origin_bound, uint32_t flags, const float* rays, uint32_t nrays,
              uint32_t* out_hits, uint32_t* out_extra, uint32_t* slot_fp, int nthreads) {
    return orc_trace_ex(tris, perm, cbox, cref, root_ref, depth, R, mode, masks, codebook, cidx, placed, lut,
                        origin_bound, flags, rays, nrays, out_hits, out_extra, slot_fp, nthreads, 0, NULL, 0);
}

/* As orc_trace, with the ray mask taken from the table at R (rm_kind 0), the
 * table at 2R (1, lut2 from orc_raymask_lut2) or the ideal mask (2), and masks
 * with more than test_max set bits untested (0 = R^3 - 1: only full masks). */
int orc_trace_ex(const float* tris, const uint32_t* perm, const float* cbox, const uint32_t* cref,
                 uint32_t root_ref, uint32_t depth, uint32_t R, uint32_t mode, const uint64_t* masks,
                 const uint64_t* codebook, const uint16_t* cidx, const uint8_t* placed, const uint64_t* lut,
                 float origin_bound, uint32_t flags, const float* rays, uint32_t nrays,
                 uint32_t* out_hits, uint32_t* out_extra, uint32_t* slot_fp, int nthreads,
                 uint32_t rm_kind, const uint64_t* lut2, uint32_t test_max) {
    if (rm_kind > 2 || (rm_kind == 1 && !lut2)) return ORC_ERR_ARG;
    if (depth + 1 > 160) return ORC_ERR_DEPTH;
    if (mode > MODE_SPARSE) return ORC_ERR_ARG;
    if (mode != MODE_NONE && (R < 1 || R > 6 || !lut)) return ORC_ERR_ARG;
    if ((mode == MODE_RAW || mode == MODE_SPARSE) && !masks) return ORC_ERR_ARG;
    if (mode == MODE_SPARSE && !placed) return ORC_ERR_ARG;
    if (mode == MODE_LUT && (!codebook || !cidx)) return ORC_ERR_ARG;
    TraceCtx C;
    C.tris = tris; C.perm = perm; C.cbox = cbox; C.cref = cref; C.root = root_ref;
    C.R = R; C.W = words_for(R ? R : 1); C.mode = mode; C.flags = flags;
    C.masks = masks; C.cb = codebook; C.cidx = cidx; C.lut = lut; C.placed = placed;
    C.origin_bound = origin_bound;
    C.slot_fp = (flags & FLAG_SHADOW) ? slot_fp : NULL;
    C.rm_kind = rm_kind;
    C.lut2 = lut2;
    C.test_max = test_max ? test_max : R * R * R - 1;
    C.cb_refs = NULL;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < (int64_t)nrays; ++i)
        trace_one(&C, &rays[8 * (size_t)i], &out_hits[4 * (size_t)i],
                  out_extra ? &out_extra[2 * (size_t)i] : NULL);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * 4-wide BVH (Sect. 3.2.4 packs four child boxes with their four masks in one
 * node). Built by collapsing the binary BVH: a 4-wide node starts from the
 * two children of a binary inner node; while it has fewer than four children
 * and one of them is a binary inner node, the inner child with the largest
 * surface area (float64; the first in child order on ties) is replaced, in
 * place, by its two children. 4-wide nodes are numbered in DFS pre-order.
 * Child c of node m: box4[24m + 6c ..] (lo xyz, hi xyz), ref4[4m + c] (leaf
 * refs unchanged, inner refs = 4-wide node index, EMPTY_REF for an unused
 * slot), src4[4m + c] = the binary child slot it came from (its mask and
 * codebook index), EMPTY_REF when unused.
 * ---------------------------------------------------------------------- */
typedef struct {
    const float* cbox; const uint32_t* cref;
    float* box4; uint32_t* ref4; uint32_t* src4;
    uint32_t n4, cap;
} Collapse;

static double slot_area(const float* cbox, uint32_t slot) {
    const float* b = &cbox[6 * (size_t)slot];
    double dx = (double)b[3] - (double)b[0], dy = (double)b[4] - (double)b[1], dz = (double)b[5] - (double)b[2];
    return 2.0 * ((dx * dy + dy * dz) + dz * dx);
}

static uint32_t collapse_rec(Collapse* K, uint32_t node2) {
    uint32_t me = K->n4++;
    uint32_t slots[4];
    int k = 2;
    slots[0] = 2u * node2;
    slots[1] = 2u * node2 + 1u;
    while (k < 4) {
        int pick = -1;
        double pick_a = 0.0;
        for (int i = 0; i < k; ++i) {
            if (K->cref[slots[i]] & LEAF_BIT) continue;
            double a = slot_area(K->cbox, slots[i]);
            if (pick < 0 || a > pick_a) { pick = i; pick_a = a; }
        }
        if (pick < 0) break;
        uint32_t inner = K->cref[slots[pick]];
        for (int i = k; i > pick + 1; --i) slots[i] = slots[i - 1];
        slots[pick] = 2u * inner;
        slots[pick + 1] = 2u * inner + 1u;
        ++k;
    }
    for (int c = 0; c < 4; ++c) {
        float* b = &K->box4[24 * (size_t)me + 6 * (size_t)c];
        if (c >= k) {
            for (int j = 0; j < 6; ++j) b[j] = 0.0f;
            K->ref4[4 * (size_t)me + c] = EMPTY_REF;
            K->src4[4 * (size_t)me + c] = EMPTY_REF;
            continue;
        }
        memcpy(b, &K->cbox[6 * (size_t)slots[c]], 6 * sizeof(float));
        K->src4[4 * (size_t)me + c] = slots[c];
        uint32_t r = K->cref[slots[c]];
        K->ref4[4 * (size_t)me + c] = (r & LEAF_BIT) ? r : collapse_rec(K, r);
    }
    return me;
}

/* Returns the number of 4-wide nodes in *n4 and the root ref in *root4
 * (a leaf or empty root stays as it is). Arrays hold at least max(n_inner,1)
 * nodes. */
int orc_bvh4_collapse(const float* cbox, const uint32_t* cref, uint32_t n_inner, uint32_t root_ref,
                      float* box4, uint32_t* ref4, uint32_t* src4, uint32_t* n4, uint32_t* root4) {
    Collapse K;
    K.cbox = cbox; K.cref = cref; K.box4 = box4; K.ref4 = ref4; K.src4 = src4; K.n4 = 0; K.cap = n_inner;
    if (root_ref == EMPTY_REF || (root_ref & LEAF_BIT) || n_inner == 0) {
        *n4 = 0;
        *root4 = root_ref;
        return ORC_OK;
    }
    *root4 = collapse_rec(&K, root_ref);
    *n4 = K.n4;
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Quantised 4-wide child boxes (not in the paper: the child-box compression of
 * compressed wide BVHs, applied to the 4-wide nodes above). Per node m and
 * axis a, over the used children only:
 *   lo_a  = min of the children's minima, hi_a = max of their maxima;
 *   dec(q, e) = float32(lo_a + float32(q * 2^e)), the decoded plane of count q
 *           at step 2^e: q * 2^e is exact in float32 (8 significant bits times
 *           a normal power of two), so the sum rounds once;
 *   e_a   = the smallest integer in [-126, 127] with 255 * 2^e_a >= hi_a - lo_a
 *           (that difference rounded to double), raised by one while some
 *           child's maximum exceeds dec(255, e_a);
 *   qlo   = floor((child min - lo_a) / 2^e_a) in [0, 255], lowered while
 *           dec(qlo) > child min; qhi = ceil((child max - lo_a) / 2^e_a) in
 *           [0, 255], raised while dec(qhi) < child max.
 * The quotients are only first guesses: child min - lo_a rounds in double when
 * the two differ greatly in magnitude, so the decoded plane itself is checked.
 * dec(0) = lo_a <= every child min and dec(255) >= every child max at the
 * final exponent, so every decoded box contains its child's box. Unused slots
 * get q = 0 and a zero decoded box. Outputs: lo[3m + a], ebias[3m + a] =
 * e_a + 127, q[24m + 6c + j] (qlo xyz, qhi xyz), dec in the layout of box4.
 * ---------------------------------------------------------------------- */
static int quant_exponent(double ext) {
    int e = -126;
    while (e < 127 && 255.0 * ldexp(1.0, e) < ext) ++e;
    return e;
}

static float quant_decode(float l, uint32_t q, float stepf) {
    const float p = (float)q * stepf;
    return l + p;
}

int orc_quantise4(const float* box4, const uint32_t* ref4, uint32_t n4, float* lo, uint8_t* ebias,
                  uint8_t* q, float* dec) {
    for (uint32_t m = 0; m < n4; ++m) {
        for (int a = 0; a < 3; ++a) {
            float l = INFINITY, h = -INFINITY;
            for (int c = 0; c < 4; ++c) {
                if (ref4[4 * (size_t)m + c] == EMPTY_REF) continue;
                const float* b = &box4[24 * (size_t)m + 6 * (size_t)c];
                if (b[a] < l) l = b[a];
                if (b[3 + a] > h) h = b[3 + a];
            }
            if (l > h) { l = 0.0f; h = 0.0f; }  /* no used child */
            int e = quant_exponent((double)h - (double)l);
            /* raise the exponent until the largest count reaches every child maximum */
            while (e < 127 && quant_decode(l, 255u, (float)ldexp(1.0, e)) < h) ++e;
            const double step = ldexp(1.0, e);
            const float stepf = (float)step;
            lo[3 * (size_t)m + a] = l;
            ebias[3 * (size_t)m + a] = (uint8_t)(e + 127);
            for (int c = 0; c < 4; ++c) {
                const size_t k = 24 * (size_t)m + 6 * (size_t)c;
                if (ref4[4 * (size_t)m + c] == EMPTY_REF) {
                    q[k + a] = 0; q[k + 3 + a] = 0;
                    dec[k + a] = 0.0f; dec[k + 3 + a] = 0.0f;
                    continue;
                }
                const float bl = box4[k + a], bh = box4[k + 3 + a];
                double ql = floor(((double)bl - (double)l) / step);
                double qh = ceil(((double)bh - (double)l) / step);
                if (ql < 0.0) ql = 0.0;
                if (ql > 255.0) ql = 255.0;
                if (qh < 0.0) qh = 0.0;
                if (qh > 255.0) qh = 255.0;
                uint32_t il = (uint32_t)ql, ih = (uint32_t)qh;
                while (il > 0 && quant_decode(l, il, stepf) > bl) --il;
                while (ih < 255 && quant_decode(l, ih, stepf) < bh) ++ih;
                q[k + a] = (uint8_t)il;
                q[k + 3 + a] = (uint8_t)ih;
                dec[k + a] = quant_decode(l, il, stepf);
                dec[k + 3 + a] = quant_decode(l, ih, stepf);
            }
        }
    }
    return ORC_OK;
}

typedef struct {
    TraceCtx base;
    const float* box4; const uint32_t* ref4; const uint32_t* src4;
} Trace4Ctx;

/* Alg. 4 on the 4-wide BVH: every used child slot gets a slab test and, when
 * it hits, the mask test of its binary slot; surviving children are visited
 * nearest t0 first (the lower child on equal t0), the others stacked with
 * their t0 and dropped on pop when t0 > best_t. */
/* deepest (optional): the most entries the stack holds while a popped entry is being visited --
 * the far children waiting beneath the current node, i.e. the stack a traversal that keeps the
 * current node out of its stack needs for this ray */
static void trace4_one(const Trace4Ctx* T, const float* ray, uint32_t* hit, uint32_t* extra,
                       uint32_t* deepest) {
    const TraceCtx* C = &T->base;
    uint32_t box_tests = 0, tri_tests = 0, mask_tests = 0, mask_culls = 0, most = 0;
    uint32_t best = NO_HIT;
    float best_t = INFINITY;
    if (ray_valid(ray) && C->root != EMPTY_REF) {
        const float o[3] = {ray[0], ray[1], ray[2]};
        const float d[3] = {ray[4], ray[5], ray[6]};
        const float tmin = ray[3];
        float inv[3] = {1.0f / d[0], 1.0f / d[1], 1.0f / d[2]};
        best_t = ray[7];
        int use_mask = (C->mode != MODE_NONE) && (C->flags & (FLAG_CULL | FLAG_SHADOW));
        if (use_mask) {
            float mo = max3f(fabsf(o[0]), fabsf(o[1]), fabsf(o[2]));
            if (mo > C->origin_bound) use_mask = 0;
        }
        int cull = (C->flags & FLAG_CULL) != 0;
        uint32_t st_ref[256];
        float st_t[256];
        int sp = 0;
        st_ref[sp] = C->root; st_t[sp] = tmin; ++sp;
        while (sp > 0) {
            --sp;
            uint32_t ref = st_ref[sp];
            float tn = st_t[sp];
            if (tn > best_t) continue;
            if ((uint32_t)sp > most) most = (uint32_t)sp;
            if (ref & LEAF_BIT) {
                leaf_tests(C, ref, o, d, tmin, &best_t, &best, &tri_tests);
                continue;
            }
            int order[4], m = 0;
            float t0c[4];
            for (int c = 0; c < 4; ++c) {
                uint32_t r = T->ref4[4 * (size_t)ref + c];
                if (r == EMPTY_REF) continue;
                const float* lo = &T->box4[24 * (size_t)ref + 6 * (size_t)c];
                const float* hi = lo + 3;
                ++box_tests;
                float t0 = tmin, t1 = best_t;
                for (int j = 0; j < 3; ++j) {
                    /* near bound first: lo for a positive direction, hi for a negative one */
                    int neg = signbit(inv[j]) != 0;
                    float a = ((neg ? hi[j] : lo[j]) - o[j]) * inv[j];
                    float b = ((neg ? lo[j] : hi[j]) - o[j]) * inv[j];
                    b = b * 0x1.000006p0f;
                    t0 = (a > t0) ? a : t0;
                    t1 = (b < t1) ? b : t1;
                }
                if (!(t0 <= t1)) continue;
                if (use_mask && mask_test(C, T->src4[4 * (size_t)ref + c], lo, hi, o, d, t0, t1, &mask_tests,
                                          &mask_culls) && cull)
                    continue;
                /* insert c by t0, after children with an equal or smaller t0 */
                int i = m++;
                while (i > 0 && t0c[i - 1] > t0) { order[i] = order[i - 1]; t0c[i] = t0c[i - 1]; --i; }
                order[i] = c;
                t0c[i] = t0;
            }
            for (int i = m - 1; i >= 0; --i) {
                st_ref[sp] = T->ref4[4 * (size_t)ref + order[i]];
                st_t[sp] = t0c[i];
                ++sp;
            }
        }
    }
    float tout = (best == NO_HIT) ? INFINITY : best_t;
    hit[0] = best;
    memcpy(&hit[1], &tout, 4);
    hit[2] = box_tests;
    hit[3] = tri_tests;
    if (extra) { extra[0] = mask_tests; extra[1] = mask_culls; }
    if (deepest) *deepest = most;
}

int orc_trace4(const float* tris, const uint32_t* perm, const float* box4, const uint32_t* ref4,
               const uint32_t* src4, uint32_t root4, uint32_t depth, uint32_t R, uint32_t mode,
               const uint64_t* masks, const uint64_t* codebook, const uint16_t* cidx, const uint8_t* placed,
               const uint64_t* lut, float origin_bound, uint32_t flags, const float* rays, uint32_t nrays,
               uint32_t* out_hits, uint32_t* out_extra, uint32_t* slot_fp, int nthreads,
               uint32_t* out_deepest, uint32_t test_max, uint32_t* out_cb_refs) {
    if (3 * depth + 1 > 256) return ORC_ERR_DEPTH;
    if (mode > MODE_SPARSE) return ORC_ERR_ARG;
    if (mode != MODE_NONE && (R < 1 || R > 6 || !lut)) return ORC_ERR_ARG;
    if ((mode == MODE_RAW || mode == MODE_SPARSE) && !masks) return ORC_ERR_ARG;
    if (mode == MODE_SPARSE && !placed) return ORC_ERR_ARG;
    if (mode == MODE_LUT && (!codebook || !cidx)) return ORC_ERR_ARG;
    Trace4Ctx T;
    TraceCtx* C = &T.base;
    C->tris = tris; C->perm = perm; C->cbox = NULL; C->cref = NULL; C->root = root4;
    C->R = R; C->W = words_for(R ? R : 1); C->mode = mode; C->flags = flags;
    C->masks = masks; C->cb = codebook; C->cidx = cidx; C->lut = lut; C->placed = placed;
    C->origin_bound = origin_bound;
    C->slot_fp = (flags & FLAG_SHADOW) ? slot_fp : NULL;
    C->rm_kind = 0;
    C->lut2 = NULL;
    C->test_max = test_max ? test_max : R * R * R - 1;
    C->cb_refs = (mode == MODE_LUT) ? out_cb_refs : NULL;
    T.box4 = box4; T.ref4 = ref4; T.src4 = src4;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < (int64_t)nrays; ++i)
        trace4_one(&T, &rays[8 * (size_t)i], &out_hits[4 * (size_t)i],
                   out_extra ? &out_extra[2 * (size_t)i] : NULL, out_deepest ? &out_deepest[i] : NULL);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * 2-D bit table (Sect. 3.2.2, note on the two LUTs): bit (key, k) is 1 iff
 * the ray mask LUT[key] and codebook entry k share a set bit, so a
 * compressed mask test becomes one bit fetch. Row key holds K bits in K/32
 * 32-bit words, entry k at bit k % 32 of word k / 32.
 * ---------------------------------------------------------------------- */
int orc_bit_table(const uint64_t* lut, uint32_t R, const uint64_t* cb, uint32_t K, uint32_t* out) {
    if (R < 1 || R > 6 || K == 0 || K % 32) return ORC_ERR_ARG;
    uint32_t W = words_for(R);
    size_t keys = (size_t)R * R * R * R * R * R;
    for (size_t key = 0; key < keys; ++key) {
        uint32_t* row = &out[key * (K / 32)];
        for (uint32_t w = 0; w < K / 32; ++w) row[w] = 0;
        for (uint32_t k = 0; k < K; ++k) {
            uint64_t any = 0;
            for (uint32_t w = 0; w < W; ++w) any |= lut[key * W + w] & cb[(size_t)k * W + w];
            if (any) row[k / 32] |= 1u << (k % 32);
        }
    }
    return ORC_OK;
}

/* Closest hit by scanning every triangle with the same triangle test and
 * tie rule; no hierarchy. out[i] = (id, t bits). */
int orc_brute_closest(const float* tris, uint32_t n, const float* rays, uint32_t nrays,
                      uint32_t* out, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < (int64_t)nrays; ++i) {
        const float* ray = &rays[8 * (size_t)i];
        uint32_t best = NO_HIT;
        float best_t = INFINITY;
        if (ray_valid(ray)) {
            const float o[3] = {ray[0], ray[1], ray[2]};
            const float d[3] = {ray[4], ray[5], ray[6]};
            float tmin = ray[3];
            best_t = ray[7];
            for (uint32_t id = 0; id < n; ++id) {
                const float* v = &tris[9 * (size_t)id];
                float e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
                float e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
                float P[3], Q[3], S[3];
                cross3(d, e2, P);
                float det = dot3(e1, P);
                if (det == 0.0f) continue;
                float idet = 1.0f / det;
                S[0] = o[0] - v[0]; S[1] = o[1] - v[1]; S[2] = o[2] - v[2];
                float u = dot3(S, P) * idet;
                if (u < 0.0f || u > 1.0f) continue;
                cross3(S, e1, Q);
                float vv = dot3(d, Q) * idet;
                if (vv < 0.0f || u + vv > 1.0f) continue;
                float t = dot3(e2, Q) * idet;
                if (t < tmin || t > best_t) continue;
                if (t < best_t || (t == best_t && id < best)) { best_t = t; best = id; }
            }
        }
        float tout = (best == NO_HIT) ? INFINITY : best_t;
        out[2 * (size_t)i] = best;
        memcpy(&out[2 * (size_t)i + 1], &tout, 4);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * 5. Compression LUT (Sect. 3.2.2, Eq. 2): importance of a node's mask is
 *    SA(N) * O_m(N) / R^3 (O_m = set bits); equal patterns add their
 *    importances in ascending slot order. The codebook holds the K-1 most
 *    important patterns other than the full mask (importance descending,
 *    then value ascending), plus the full mask, padded with full masks to K,
 *    then sorted by (set bits ascending, value ascending) so that the lowest
 *    conservative index is the tightest (Sect. 3.2.3). Value order reads the
 *    mask as an unsigned integer whose last word is most significant.
 * ---------------------------------------------------------------------- */
static uint32_t g_W;  /* word count for the qsort comparators */

static int cmp_value(const uint64_t* a, const uint64_t* b) {
    for (int w = (int)g_W - 1; w >= 0; --w) {
        if (a[w] < b[w]) return -1;
        if (a[w] > b[w]) return 1;
    }
    return 0;
}

typedef struct { const uint64_t* m; uint32_t slot; double imp; uint32_t pc; } Item;

static int cmp_slot_by_value(const void* x, const void* y) {
    const Item* a = (const Item*)x;
    const Item* b = (const Item*)y;
    int c = cmp_value(a->m, b->m);
    if (c) return c;
    return (a->slot < b->slot) ? -1 : (a->slot > b->slot);
}

static int cmp_importance(const void* x, const void* y) {
    const Item* a = (const Item*)x;
    const Item* b = (const Item*)y;
    if (a->imp > b->imp) return -1;
    if (a->imp < b->imp) return 1;
    return cmp_value(a->m, b->m);
}

static int cmp_pop_value(const void* x, const void* y) {
    const Item* a = (const Item*)x;
    const Item* b = (const Item*)y;
    if (a->pc != b->pc) return (a->pc < b->pc) ? -1 : 1;
    return cmp_value(a->m, b->m);
}

static uint32_t popc(const uint64_t* m, uint32_t W) {
    uint32_t c = 0;
    for (uint32_t w = 0; w < W; ++w) c += (uint32_t)__builtin_popcountll(m[w]);
    return c;
}

static void full_mask(uint32_t R, uint64_t* m) {
    uint32_t W = words_for(R), R3 = R * R * R;
    for (uint32_t w = 0; w < W; ++w) m[w] = 0;
    for (uint32_t b = 0; b < R3; ++b) m[b >> 6] |= 1ull << (b & 63);
}

/* boxes: [S][6] (lo xyz, hi xyz) of each slot. */
int orc_codebook(const uint64_t* masks, const float* boxes, uint32_t S, uint32_t R, uint32_t K,
                 uint64_t* cb) {
    if (R < 1 || R > 6 || K < 1) return ORC_ERR_ARG;
    uint32_t W = words_for(R);
    g_W = W;
    uint64_t full[4];
    full_mask(R, full);
    Item* it = (Item*)malloc((size_t)(S ? S : 1) * sizeof(Item));
    if (!it) return ORC_ERR_OOM;
    for (uint32_t s = 0; s < S; ++s) {
        const float* b = &boxes[6 * (size_t)s];
        double dx = (double)b[3] - (double)b[0];
        double dy = (double)b[4] - (double)b[1];
        double dz = (double)b[5] - (double)b[2];
        double sa = 2.0 * ((dx * dy + dy * dz) + dz * dx);
        it[s].m = &masks[(size_t)s * W];
        it[s].slot = s;
        it[s].pc = popc(it[s].m, W);
        it[s].imp = (sa * (double)it[s].pc) / (double)(R * R * R);
    }
    qsort(it, S, sizeof(Item), cmp_slot_by_value);
    /* collapse equal patterns; sums run in ascending slot order */
    uint32_t nd = 0;
    for (uint32_t i = 0; i < S;) {
        uint32_t j = i;
        double sum = 0.0;
        while (j < S && cmp_value(it[j].m, it[i].m) == 0) { sum += it[j].imp; ++j; }
        if (cmp_value(it[i].m, full) != 0) {
            it[nd] = it[i];
            it[nd].imp = sum;
            ++nd;
        }
        i = j;
    }
    qsort(it, nd, sizeof(Item), cmp_importance);
    uint32_t take = nd < K - 1 ? nd : K - 1;
    Item* sel = (Item*)malloc((size_t)K * sizeof(Item));
    if (!sel) { free(it); return ORC_ERR_OOM; }
    for (uint32_t i = 0; i < take; ++i) sel[i] = it[i];
    for (uint32_t i = take; i < K; ++i) { sel[i].m = full; sel[i].pc = popc(full, W); sel[i].imp = 0; sel[i].slot = 0; }
    qsort(sel, K, sizeof(Item), cmp_pop_value);
    for (uint32_t k = 0; k < K; ++k)
        for (uint32_t w = 0; w < W; ++w) cb[(size_t)k * W + w] = sel[k].m[w];
    free(sel);
    free(it);
    return ORC_OK;
}

/* Requirement LUTs (Sect. 3.2.3): table i, row p, bit k is set iff codebook
 * entry k has every bit of p in its chunk i, chunk i being mask bits
 * [8i, 8i+8). Rows are K bits, K a multiple of 64. */
static inline uint32_t chunk8(const uint64_t* m, uint32_t i) {
    uint32_t bit = 8 * i;
    return (uint32_t)((m[bit >> 6] >> (bit & 63)) & 0xFFu);
}

int orc_req_luts(const uint64_t* cb, uint32_t K, uint32_t R, uint64_t* req) {
    if (K % 64 || R < 1 || R > 6) return ORC_ERR_ARG;
    uint32_t W = words_for(R), nch = (R * R * R + 7) / 8, KW = K / 64;
    for (uint32_t i = 0; i < nch; ++i)
        for (uint32_t p = 0; p < 256; ++p) {
            uint64_t* row = &req[((size_t)i * 256 + p) * KW];
            for (uint32_t w = 0; w < KW; ++w) row[w] = 0;
            for (uint32_t k = 0; k < K; ++k)
                if ((chunk8(&cb[(size_t)k * W], i) & p) == p) row[k >> 6] |= 1ull << (k & 63);
        }
    return ORC_OK;
}

/* Alg. 3: AND the rows selected by each 8-bit chunk, return the lowest set bit. */
int orc_alg3(const uint64_t* masks, uint32_t S, const uint64_t* req, uint32_t K, uint32_t R,
             uint16_t* out_idx) {
    if (K % 64 || K > 65536) return ORC_ERR_ARG;
    uint32_t W = words_for(R), nch = (R * R * R + 7) / 8, KW = K / 64;
    uint64_t* acc = (uint64_t*)malloc((size_t)KW * sizeof(uint64_t));
    if (!acc) return ORC_ERR_OOM;
    for (uint32_t s = 0; s < S; ++s) {
        const uint64_t* m = &masks[(size_t)s * W];
        for (uint32_t w = 0; w < KW; ++w) acc[w] = req[(size_t)chunk8(m, 0) * KW + w];
        for (uint32_t i = 1; i < nch; ++i) {
            const uint64_t* row = &req[((size_t)i * 256 + chunk8(m, i)) * KW];
            for (uint32_t w = 0; w < KW; ++w) acc[w] &= row[w];
        }
        uint32_t idx = 0xFFFFu;
        for (uint32_t w = 0; w < KW; ++w)
            if (acc[w]) { idx = w * 64 + (uint32_t)__builtin_ctzll(acc[w]); break; }
        out_idx[s] = (uint16_t)idx;
    }
    free(acc);
    return ORC_OK;
}

/* The brute-force search named in Sect. 3.2.3: scan all K entries, keep the
 * superset with the fewest set bits (first one on ties). */
int orc_naive_search(const uint64_t* masks, uint32_t S, const uint64_t* cb, uint32_t K, uint32_t R,
                     uint16_t* out_idx) {
    uint32_t W = words_for(R);
    for (uint32_t s = 0; s < S; ++s) {
        const uint64_t* m = &masks[(size_t)s * W];
        uint32_t best = 0xFFFFu, best_pc = 0xFFFFFFFFu;
        for (uint32_t k = 0; k < K; ++k) {
            const uint64_t* c = &cb[(size_t)k * W];
            int sup = 1;
            for (uint32_t w = 0; w < W; ++w)
                if ((m[w] & ~c[w]) != 0) { sup = 0; break; }
            if (!sup) continue;
            uint32_t pc = popc(c, W);
            if (pc < best_pc) { best_pc = pc; best = k; }
        }
        out_idx[s] = (uint16_t)best;
    }
    return ORC_OK;
}

/* One triangle against one box, for closed-form checks: out[W] = bits. */
int orc_voxelize_tri(const float* tri, const float* lo, const float* hi, uint32_t R, float delta,
                     uint64_t* out) {
    if (R < 1 || R > 6) return ORC_ERR_ARG;
    uint32_t W = words_for(R);
    for (uint32_t w = 0; w < W; ++w) out[w] = 0;
    voxelize_tri(tri, lo, hi, R, delta, out);
    return ORC_OK;
}

/* Alg. 1 alone: ray mask of box (lo, hi) for the segment [t0, t1] of ray
 * (o, d), read from the LUT. out[W]. */
int orc_ray_mask(const float* lo, const float* hi, const float* o, const float* d, float t0,
                 float t1, uint32_t R, const uint64_t* lut, uint64_t* out) {
    if (R < 1 || R > 6) return ORC_ERR_ARG;
    int cb_[3], ce_[3];
    raymask_key_cells(lo, hi, o, d, t0, R, cb_);
    raymask_key_cells(lo, hi, o, d, t1, R, ce_);
    size_t key = (((((size_t)cb_[0] * R + cb_[1]) * R + cb_[2]) * R + ce_[0]) * R + ce_[1]) * R + ce_[2];
    uint32_t W = words_for(R);
    for (uint32_t w = 0; w < W; ++w) out[w] = lut[key * W + w];
    return ORC_OK;
}

/* Object masks of selected child slots only: out[i*W..] for slots[i]. */
int orc_slot_masks(const float* tris, const uint32_t* perm, const float* cbox, const uint32_t* cref,
                   const uint32_t* range, const uint32_t* slots, uint32_t nslots, uint32_t R, float delta,
                   uint64_t* out, int nthreads) {
    if (R < 1 || R > 6) return ORC_ERR_ARG;
    uint32_t W = words_for(R);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t i = 0; i < (int64_t)nslots; ++i) {
        uint32_t s = slots[i];
        uint64_t* m = &out[(size_t)i * W];
        for (uint32_t w = 0; w < W; ++w) m[w] = 0;
        const float* bx = &cbox[12 * (size_t)(s >> 1) + 6 * (size_t)(s & 1)];
        uint32_t first, count;
        slot_range(cref, range, s, &first, &count);
        for (uint32_t j = first; j < first + count; ++j)
            voxelize_tri(&tris[9 * (size_t)perm[j]], bx, bx + 3, R, delta, m);
    }
    return ORC_OK;
}
