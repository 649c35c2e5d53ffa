/*
 * CPU oracle for the hybrid depth-of-field pass (Tan, Chua, Biette & Bhojan,
 * "A Hybrid System for Real-Time Rendering of Depth of Field Effect in Games").
 *
 * TEST INFRASTRUCTURE ONLY: see oracle.h.  Build with
 *     gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared
 * Plain sequential loops in binary32; OpenMP only splits independent pixels
 * or rays, so results do not depend on the thread count.
 *
 * Stage names (A1..A14) follow the order in which the paper's section 3
 * describes the pass: post-process branch (3.1), ray-trace branch (3.2),
 * composite (3.3).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_SQRT2 1.41421356237f   /* diagonal of one pixel (3.1.1, 3.3) */
#define LEAF_BIT 0x80000000u

static int g_threads = 1;

void orc_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int orc_threads(void) { return g_threads; }

/* ------------------------------------------------------------------------ */
/* small scalar helpers (compare-select, so NaN and signed zero are fixed)   */
/* ------------------------------------------------------------------------ */

static float fmin_cs(float a, float b) { return b < a ? b : a; }
static float fmax_cs(float a, float b) { return b > a ? b : a; }
static float sat(float x) { return x > 0.0f ? (x < 1.0f ? x : 1.0f) : 0.0f; }
static float clampf(float x, float lo, float hi) { return x < lo ? lo : (x > hi ? hi : x); }
static int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }
static float lerpf(float a, float b, float t) { return a + (b - a) * t; }
static float luma(float r, float g, float b) { return (0.2126f * r + 0.7152f * g) + 0.0722f * b; }

/* ------------------------------------------------------------------------ */
/* Thin-lens quantities (section 3.3, eq. 6)                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    float a;        /* aperture diameter f/N */
    float tanx, tany;
    float cock;     /* CoC(z) = cock * |1 - d/z| in full-res pixels */
    float znb, zfb; /* zone of focus, eq. (6) with w_i = image width */
    float ramp;     /* width of the near/far transition (3.2.2) */
    float half_a;
    float ju, jv;   /* camera jitter as an offset of normalised image coordinates */
} lensq;

static lensq lens_quantities(const orc_lens *l, int W, int H)
{
    lensq q;
    float f = l->focal, d = l->focus, ws = l->sensor;
    q.a = f / l->fnum;
    /* Pixel footprint follows the sensor at the focused image distance
     * v = f d / (d - f): tan of the half field = (w_s / 2) / v. */
    q.tanx = (ws * (d - f)) / ((2.0f * f) * d);
    q.tany = q.tanx * ((float)H / (float)W);
    /* Thin-lens blur diameter a f |z - d| / (z (d - f)) on the sensor, in
     * pixels of an image w_i wide: setting it to sqrt(2) gives both bounds of
     * eq. (6). */
    q.cock = ((q.a * f) / (d - f)) * ((float)W / ws);
    float g = (OR_SQRT2 * (d - f)) * (ws / (float)W);
    float af = q.a * f;
    q.znb = (af * d) / (af + g);
    q.zfb = (af > g) ? (af * d) / (af - g) : INFINITY;
    q.ramp = 2.0f * (d - q.znb);
    q.half_a = q.a * 0.5f;
    q.ju = 0.0f;
    q.jv = 0.0f;
    return q;
}

static float coc_of(const lensq *q, float d, float z) { return q->cock * fabsf(1.0f - d / z); }

float orc_coc(const orc_lens *lens, int32_t width, float z)
{
    lensq q = lens_quantities(lens, width, width);
    return coc_of(&q, lens->focus, z);
}

int orc_zone(const orc_lens *lens, int32_t width, float *z_near, float *z_far)
{
    if (!lens || width <= 0) return -1;
    lensq q = lens_quantities(lens, width, width);
    *z_near = q.znb;
    *z_far = q.zfb;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Counter hash for lens samples: PCG-RXS-M-XS 32-bit hash as published by   */
/* Jarzynski & Olano, "Hash Functions for GPU Rendering", JCGT 2020.         */
/* ------------------------------------------------------------------------ */

static uint32_t pcg_hash(uint32_t v)
{
    uint32_t state = v * 747796405u + 2891336453u;
    uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

typedef struct {
    int blades;
    float apothem;
    float nx[16], ny[16];
} aperture;

static aperture make_aperture(int blades, float rot)
{
    aperture ap;
    ap.blades = blades;
    ap.apothem = 1.0f;
    if (blades >= 3) {
        const double pi = 3.14159265358979323846;
        ap.apothem = (float)cos(pi / blades);
        for (int i = 0; i < blades; i++) {
            double th = (double)rot + pi / blades + 2.0 * pi * i / blades;
            ap.nx[i] = (float)cos(th);
            ap.ny[i] = (float)sin(th);
        }
    }
    return ap;
}

static int inside_aperture(const aperture *ap, float x, float y)
{
    if (ap->blades < 3) return x * x + y * y < 1.0f;
    for (int i = 0; i < ap->blades; i++)
        if (x * ap->nx[i] + y * ap->ny[i] > ap->apothem) return 0;
    return 1;
}

/* Section 3.2.2: random positions within the lens aperture, drawn by
 * rejection from the square [-1,1)^2 with at most 32 attempts. */
static void lens_point(const aperture *ap, uint32_t seed, uint32_t frame, uint32_t q,
                       uint32_t k, float *lx, float *ly)
{
    uint32_t h = pcg_hash(pcg_hash(pcg_hash(seed) ^ frame) ^ q);
    for (uint32_t att = 0; att < 32u; att++) {
        uint32_t a = pcg_hash(h ^ ((k << 8) | att));
        uint32_t b = pcg_hash(a);
        float x = (float)(a >> 8) * (1.0f / 8388608.0f) - 1.0f;
        float y = (float)(b >> 8) * (1.0f / 8388608.0f) - 1.0f;
        if (inside_aperture(ap, x, y)) { *lx = x; *ly = y; return; }
    }
    *lx = 0.0f;
    *ly = 0.0f;
}

int orc_lens_sample(uint32_t seed, uint32_t frame, uint32_t q, uint32_t k,
                    int32_t blades, float blade_rot, float *lx, float *ly)
{
    if (blades > 16 || (blades > 0 && blades < 3)) return -1;
    aperture ap = make_aperture(blades, blade_rot);
    lens_point(&ap, seed, frame, q, k, lx, ly);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Morton codes and the binary radix tree (the GPU-side acceleration         */
/* structure that stands in for the DXR build the paper times in 5.2)        */
/* ------------------------------------------------------------------------ */

static void tri_box(const float *v, float lo[3], float hi[3])
{
    for (int a = 0; a < 3; a++) {
        float x = v[a], y = v[3 + a], z = v[6 + a];
        float m = x;
        m = y < m ? y : m;
        m = z < m ? z : m;
        lo[a] = m;
        float M = x;
        M = y > M ? y : M;
        M = z > M ? z : M;
        hi[a] = M;
    }
}

static uint64_t spread21(uint32_t x)
{
    /* place bit i of x at bit 3i, bit by bit */
    uint64_t r = 0;
    for (int i = 0; i < 21; i++) r |= (uint64_t)((x >> i) & 1u) << (3 * i);
    return r;
}

/* LBVH key of a box: a 63-bit Morton code (21 bits per axis, x at bit 3i+2,
 * y at 3i+1, z at 3i) of its centre, quantised on cubic cells (one scale
 * 2^21 / largest extent of the centre bounds, for all axes), and bit 63 set
 * for a large box: one whose diagonal exceeds a quarter of the diagonal of
 * the centre bounds (compared squared).  The flag puts the few scene-sized
 * triangles (ground planes) under one child of the root instead of inflating
 * every box on their path. */
int orc_morton_boxes(const float *boxes, int64_t n, uint64_t *codes)
{
    if (!boxes || n <= 0 || !codes) return -1;
    float *cen = (float *)malloc(sizeof(float) * 3 * (size_t)n);
    float *diag2 = (float *)malloc(sizeof(float) * (size_t)n);
    if (!cen || !diag2) {
        free(cen);
        free(diag2);
        return -2;
    }
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; i++) {
        const float *bl = boxes + 6 * (size_t)i, *bh = bl + 3;
        for (int a = 0; a < 3; a++) {
            float c = (bl[a] + bh[a]) * 0.5f;
            cen[3 * (size_t)i + a] = c;
            lo[a] = c < lo[a] ? c : lo[a];
            hi[a] = c > hi[a] ? c : hi[a];
        }
        float dx = bh[0] - bl[0], dy = bh[1] - bl[1], dz = bh[2] - bl[2];
        diag2[i] = (dx * dx + dy * dy) + dz * dz;
    }
    float ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    float e = ext[0];
    e = ext[1] > e ? ext[1] : e;
    e = ext[2] > e ? ext[2] : e;
    float inv = e > 0.0f ? 2097152.0f / e : 0.0f;
    float large = ((ext[0] * ext[0] + ext[1] * ext[1]) + ext[2] * ext[2]) * 0.0625f;
    for (int64_t i = 0; i < n; i++) {
        uint32_t qv[3];
        for (int a = 0; a < 3; a++) {
            float t = floorf((cen[3 * (size_t)i + a] - lo[a]) * inv);
            int qi = (int)t;
            qv[a] = (uint32_t)(qi > 2097151 ? 2097151 : qi);
        }
        uint64_t flag = diag2[i] > large ? 1u : 0u;
        codes[i] = (flag << 63) | (spread21(qv[0]) << 2) | (spread21(qv[1]) << 1) | spread21(qv[2]);
    }
    free(cen);
    free(diag2);
    return 0;
}

/* Keys of the triangles' own boxes (no leaf splitting). */
int orc_morton(const orc_scene *s, uint64_t *codes)
{
    if (!s || s->ntri <= 0 || !codes) return -1;
    float *boxes = (float *)malloc(sizeof(float) * 6 * (size_t)s->ntri);
    if (!boxes) return -2;
    for (int i = 0; i < s->ntri; i++) tri_box(s->verts + 9 * (size_t)i, boxes + 6 * (size_t)i, boxes + 6 * (size_t)i + 3);
    int rc = orc_morton_boxes(boxes, s->ntri, codes);
    free(boxes);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Leaf references: early split clipping (Ernst & Greiner, "Early Split     */
/* Clipping for Bounding Volume Hierarchies", IEEE RT 2007).  A long thin    */
/* slanted triangle (a grass blade, a fence wire) fills little of its box,   */
/* so most rays that enter the box miss it.  Such a triangle becomes 2, 4 or */
/* 8 leaf references, the triangle clipped to equal slabs of its box along   */
/* the box's longest axis; each reference's box bounds its piece.            */
/* ------------------------------------------------------------------------ */

/* A triangle is thin iff the sum of its box's three face areas exceeds 8
 * times its area: (sum)^2 > 16 |e1 x e2|^2, in binary64 (deterministic; the
 * library decides with the same formula).  A thin triangle gets 2^split
 * references, any other one. */
static int ref_count(const float *v, int split)
{
    float lo[3], hi[3];
    tri_box(v, lo, hi);
    double e[3], u[3], w[3];
    for (int a = 0; a < 3; a++) {
        e[a] = (double)hi[a] - (double)lo[a];
        u[a] = (double)v[3 + a] - (double)v[a];
        w[a] = (double)v[6 + a] - (double)v[a];
    }
    double faces = (e[0] * e[1] + e[1] * e[2]) + e[2] * e[0];
    double cx = u[1] * w[2] - u[2] * w[1];
    double cy = u[2] * w[0] - u[0] * w[2];
    double cz = u[0] * w[1] - u[1] * w[0];
    double c2 = (cx * cx + cy * cy) + cz * cz;
    return (c2 > 0.0 && faces * faces > 16.0 * c2) ? 1 << split : 1;
}

int64_t orc_leaf_refs(const orc_scene *s, uint32_t *ref_off)
{
    if (!s || s->ntri <= 0 || !ref_off || s->leaf_split < 0 || s->leaf_split > 3) return -1;
    uint64_t acc = 0;
    for (int i = 0; i < s->ntri; i++) {
        ref_off[i] = (uint32_t)acc;
        acc += s->leaf_split ? (uint64_t)ref_count(s->verts + 9 * (size_t)i, s->leaf_split) : 1u;
        if (acc > 0x7fffffffu) return -1;
    }
    ref_off[s->ntri] = (uint32_t)acc;
    return (int64_t)acc;
}

/* Box of the piece of triangle v inside the slab s0 <= x_k <= s1: on axis k
 * the slab; on each other axis the range of the vertices inside the slab and
 * of the points where edges cross its planes.  A crossing point is computed
 * in binary32 and widened by 2^-20 (|edge extent| + |x|), more than its
 * rounding error, then the range is clipped to the triangle's box: every
 * point of the piece lies in the box. */
static void piece_box(const float *v, int k, float s0, float s1, const float lo[3], const float hi[3], float *out)
{
    out[k] = s0;
    out[3 + k] = s1;
    for (int m = 0; m < 3; m++) {
        if (m == k) continue;
        float pl = INFINITY, ph = -INFINITY;
        for (int i = 0; i < 3; i++) {
            float vk = v[3 * i + k];
            if (vk >= s0 && vk <= s1) {
                float x = v[3 * i + m];
                pl = x < pl ? x : pl;
                ph = x > ph ? x : ph;
            }
        }
        for (int e = 0; e < 3; e++) {
            const float *p = v + 3 * e, *q = v + 3 * ((e + 1) % 3);
            for (int c = 0; c < 2; c++) {
                float pc = c ? s1 : s0;
                if ((p[k] < pc && pc < q[k]) || (q[k] < pc && pc < p[k])) {
                    float t = (pc - p[k]) / (q[k] - p[k]);
                    float d = q[m] - p[m];
                    float x = p[m] + d * t;
                    float g = (fabsf(d) + fabsf(x)) * 9.5367431640625e-07f;
                    float xl = x - g, xh = x + g;
                    pl = xl < pl ? xl : pl;
                    ph = xh > ph ? xh : ph;
                }
            }
        }
        pl = lo[m] > pl ? lo[m] : pl;
        ph = hi[m] < ph ? hi[m] : ph;
        if (pl > ph) {
            pl = lo[m];
            ph = hi[m];
        }
        out[m] = pl;
        out[3 + m] = ph;
    }
}

int orc_ref_boxes(const orc_scene *s, const uint32_t *ref_off, float *boxes, uint32_t *ref_tri)
{
    if (!s || s->ntri <= 0 || !ref_off || !boxes || !ref_tri) return -1;
    for (int i = 0; i < s->ntri; i++) {
        const float *v = s->verts + 9 * (size_t)i;
        const uint32_t r0 = ref_off[i], nr = ref_off[i + 1] - r0;
        float lo[3], hi[3];
        tri_box(v, lo, hi);
        if (nr == 1) {
            float *o = boxes + 6 * (size_t)r0;
            for (int a = 0; a < 3; a++) { o[a] = lo[a]; o[3 + a] = hi[a]; }
            ref_tri[r0] = (uint32_t)i;
            continue;
        }
        if (nr != 2 && nr != 4 && nr != 8) return -1;
        /* nr equal slabs along the longest box axis (first one on ties) */
        float ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
        int k = 0;
        if (ext[1] > ext[k]) k = 1;
        if (ext[2] > ext[k]) k = 2;
        float q = ext[k] * (1.0f / (float)nr), sl[9];
        sl[0] = lo[k];
        sl[nr] = hi[k];
        for (uint32_t j = 1; j < nr; j++) {
            float x = lo[k] + q * (float)j;
            sl[j] = x < hi[k] ? x : hi[k];
        }
        for (uint32_t j = 0; j < nr; j++) {
            piece_box(v, k, sl[j], sl[j + 1], lo, hi, boxes + 6 * (size_t)(r0 + j));
            ref_tri[r0 + j] = (uint32_t)i;
        }
    }
    return 0;
}

typedef struct {
    uint64_t code;
    uint32_t id;
} keyed;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

static void box_union(const float *a, const float *b, float *o)
{
    for (int k = 0; k < 3; k++) {
        o[k] = b[k] < a[k] ? b[k] : a[k];
        o[3 + k] = b[3 + k] > a[3 + k] ? b[3 + k] : a[3 + k];
    }
}

/* Bit b (0 = most significant) of the 96-bit key (code << 32 | reference) of
 * leaf i: the code occupies key bits 0..63, the reference index bits 64..95. */
static int key_bit(const orc_bvh *b, uint32_t i, int bit)
{
    if (bit < 64) return (int)((b->keys[i] >> (63 - bit)) & 1u);
    return (int)((b->refs[i] >> (95 - bit)) & 1u);
}

/* Top-down: the node covering sorted leaves [first, last] splits where the
 * most significant key bit in which its first and last keys differ turns from
 * 0 to 1.  The left child is numbered by its last leaf, the right child by
 * its first leaf, the root is 0 (Karras 2012 numbering). */
static void build_rec(orc_bvh *b, uint32_t first, uint32_t last, uint32_t index)
{
    int bit = 0;
    while (key_bit(b, first, bit) == key_bit(b, last, bit)) bit++;
    uint32_t split = first;
    while (split + 1 <= last && key_bit(b, split + 1, bit) == 0) split++;
    uint32_t l, r;
    if (split == first) {
        l = split | LEAF_BIT;
        b->parent[(b->nleaf - 1) + split] = index;
    } else {
        l = split;
        b->parent[split] = index;
        build_rec(b, first, split, split);
    }
    if (split + 1 == last) {
        r = (split + 1) | LEAF_BIT;
        b->parent[(b->nleaf - 1) + split + 1] = index;
    } else {
        r = split + 1;
        b->parent[split + 1] = index;
        build_rec(b, split + 1, last, split + 1);
    }
    b->left[index] = l;
    b->right[index] = r;
    const float *lb = (l & LEAF_BIT) ? b->leaf_bounds + 6 * (size_t)(l & ~LEAF_BIT) : b->bounds + 6 * (size_t)l;
    const float *rb = (r & LEAF_BIT) ? b->leaf_bounds + 6 * (size_t)(r & ~LEAF_BIT) : b->bounds + 6 * (size_t)r;
    box_union(lb, rb, b->bounds + 6 * (size_t)index);
}

int orc_build_bvh(const orc_scene *s, orc_bvh *b)
{
    if (!s || !b || s->ntri <= 0) return -1;
    int status = 0;
    uint32_t *ref_off = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)s->ntri + 1));
    float *boxes = NULL;
    uint32_t *ref_tri = NULL;
    uint64_t *codes = NULL;
    keyed *kv = NULL;
    if (!ref_off) return -2;
    const int64_t n = orc_leaf_refs(s, ref_off);
    if (n <= 0 || n != b->nleaf) { status = -1; goto done; }
    boxes = (float *)malloc(sizeof(float) * 6 * (size_t)n);
    ref_tri = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    codes = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    kv = (keyed *)malloc(sizeof(keyed) * (size_t)n);
    if (!boxes || !ref_tri || !codes || !kv) { status = -2; goto done; }
    if (orc_ref_boxes(s, ref_off, boxes, ref_tri) != 0) { status = -1; goto done; }
    if (orc_morton_boxes(boxes, n, codes) != 0) { status = -2; goto done; }
    for (int64_t i = 0; i < n; i++) { kv[i].code = codes[i]; kv[i].id = (uint32_t)i; }
    qsort(kv, (size_t)n, sizeof(keyed), cmp_keyed);
    for (int64_t i = 0; i < n; i++) {
        const uint32_t r = kv[i].id;
        b->keys[i] = kv[i].code;
        b->refs[i] = r;
        b->ids[i] = ref_tri[r];
        memcpy(b->leaf_bounds + 6 * (size_t)i, boxes + 6 * (size_t)r, sizeof(float) * 6);
    }
    b->parent[0] = ~0u;
    if (n > 1) build_rec(b, 0, (uint32_t)n - 1, 0);
done:
    free(ref_off);
    free(boxes);
    free(ref_tri);
    free(codes);
    free(kv);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Closest hit: watertight ray/triangle test of Woop, Benthin & Wald,        */
/* "Watertight Ray/Triangle Intersection", JCGT 2013, two-sided.             */
/* ------------------------------------------------------------------------ */

typedef struct {
    float o[3], d[3];
    int kx, ky, kz;
    float sx, sy, sz;
} wray;

static wray make_wray(const float o[3], const float d[3])
{
    wray r;
    memcpy(r.o, o, sizeof(r.o));
    memcpy(r.d, d, sizeof(r.d));
    float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    if (d[kz] < 0.0f) { int t = kx; kx = ky; ky = t; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.sx = d[kx] / d[kz];
    r.sy = d[ky] / d[kz];
    r.sz = 1.0f / d[kz];
    return r;
}

/* Returns 1 and the distance along the ray on a hit with t > 0. */
static int tri_hit(const wray *r, const float *v, float *tout)
{
    float A[3], B[3], C[3];
    for (int a = 0; a < 3; a++) {
        A[a] = v[a] - r->o[a];
        B[a] = v[3 + a] - r->o[a];
        C[a] = v[6 + a] - r->o[a];
    }
    float Ax = A[r->kx] - r->sx * A[r->kz];
    float Ay = A[r->ky] - r->sy * A[r->kz];
    float Bx = B[r->kx] - r->sx * B[r->kz];
    float By = B[r->ky] - r->sy * B[r->kz];
    float Cx = C[r->kx] - r->sx * C[r->kz];
    float Cy = C[r->ky] - r->sy * C[r->kz];
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        /* edge case: redo the three 2D edge functions in binary64 */
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0;
    float det = U + V + W;
    if (det == 0.0f) return 0;
    float Az = r->sz * A[r->kz];
    float Bz = r->sz * B[r->kz];
    float Cz = r->sz * C[r->kz];
    float T = (U * Az + V * Bz) + W * Cz;
    float t = T / det;
    if (!(t > 0.0f) || !(t < INFINITY)) return 0;
    *tout = t;
    return 1;
}

/* Total order on hits: smaller t, then smaller original triangle id. */
static void consider(const orc_scene *s, const wray *r, uint32_t id, float *tb, int32_t *ib)
{
    float t;
    if (tri_hit(r, s->verts + 9 * (size_t)id, &t)) {
        if (t < *tb || (t == *tb && (*ib < 0 || id < (uint32_t)*ib))) {
            *tb = t;
            *ib = (int32_t)id;
        }
    }
}

/* Slab test in binary64 with a relative allowance, so that it never rejects
 * a box whose contents could still produce a closer (or equal) hit. */
static int box_hit(const float *bx, const double o[3], const double inv[3], const int zero[3],
                   double tbest)
{
    double tn = -INFINITY, tf = INFINITY;
    for (int a = 0; a < 3; a++) {
        if (zero[a]) {
            if (o[a] < bx[a] || o[a] > bx[3 + a]) return 0;
            continue;
        }
        double t0 = (bx[a] - o[a]) * inv[a], t1 = (bx[3 + a] - o[a]) * inv[a];
        if (t0 > t1) { double t = t0; t0 = t1; t1 = t; }
        if (t0 > tn) tn = t0;
        if (t1 < tf) tf = t1;
    }
    double slack = 1e-6 * (fabs(tn) + fabs(tf)) + 1e-9;
    if (tn > tf + slack) return 0;
    if (tf < -slack) return 0;
    if (tn > tbest + 1e-4 * fabs(tbest) + 1e-7) return 0;
    return 1;
}

static void trace_rec(const orc_scene *s, const orc_bvh *b, const wray *r,
                      const double o[3], const double inv[3], const int zero[3],
                      uint32_t node, float *tb, int32_t *ib)
{
    uint32_t ch[2] = {b->left[node], b->right[node]};
    for (int c = 0; c < 2; c++) {
        uint32_t x = ch[c];
        const float *bx = (x & LEAF_BIT) ? b->leaf_bounds + 6 * (size_t)(x & ~LEAF_BIT)
                                         : b->bounds + 6 * (size_t)x;
        if (!box_hit(bx, o, inv, zero, (double)*tb)) continue;
        if (x & LEAF_BIT) {
            consider(s, r, b->ids[x & ~LEAF_BIT], tb, ib);
        } else {
            trace_rec(s, b, r, o, inv, zero, x, tb, ib);
        }
    }
}

static void closest(const orc_scene *s, const orc_bvh *b, const float o[3], const float d[3],
                    int32_t *hit, float *tout)
{
    wray r = make_wray(o, d);
    float tb = INFINITY;
    int32_t ib = -1;
    if (!b) {
        for (int i = 0; i < s->ntri; i++) consider(s, &r, (uint32_t)i, &tb, &ib);
    } else if (s->ntri == 1) {
        consider(s, &r, 0u, &tb, &ib);
    } else {
        double od[3], inv[3];
        int zero[3];
        for (int a = 0; a < 3; a++) {
            od[a] = o[a];
            zero[a] = d[a] == 0.0f;
            inv[a] = zero[a] ? 0.0 : 1.0 / (double)d[a];
        }
        trace_rec(s, b, &r, od, inv, zero, 0u, &tb, &ib);
    }
    *hit = ib;
    *tout = tb;
}

int orc_closest_hit(const orc_scene *s, const orc_bvh *b, int64_t nrays,
                    const float *org, const float *dir, int32_t *hit, float *t)
{
    if (!s || s->ntri <= 0 || nrays < 0) return -1;
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads)
    for (int64_t i = 0; i < nrays; i++) closest(s, b, org + 3 * i, dir + 3 * i, hit + i, t + i);
    return 0;
}

/* Lambert shading of a hit (the synthetic scenes' material): two-sided
 * geometric normal turned to face the ray, one directional light plus an
 * ambient term. */
static void shade(const orc_scene *s, uint32_t id, const float d[3], float rgb[3], float nrm[3])
{
    const float *v = s->verts + 9 * (size_t)id;
    float e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    float e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    float n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                  e1[0] * e2[1] - e1[1] * e2[0]};
    float len = sqrtf((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
    n[0] = n[0] / len; n[1] = n[1] / len; n[2] = n[2] / len;
    if ((n[0] * d[0] + n[1] * d[1]) + n[2] * d[2] > 0.0f) {
        n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2];
    }
    float ndl = -((n[0] * s->light_dir[0] + n[1] * s->light_dir[1]) + n[2] * s->light_dir[2]);
    if (!(ndl > 0.0f)) ndl = 0.0f;
    const float *al = s->albedo + 3 * (size_t)id;
    for (int c = 0; c < 3; c++) rgb[c] = al[c] * (s->light_rad[c] * ndl + s->ambient[c]);
    if (nrm) { nrm[0] = n[0]; nrm[1] = n[1]; nrm[2] = n[2]; }
}

/* Sub-pixel camera jitter (3.1.2): the frame's sample positions move by
 * (jitter[0], jitter[1]) full-res pixels to the right and down.  As an offset
 * of the normalised image coordinates it is the same on every grid. */
static void set_jitter(lensq *q, const orc_camera *c)
{
    q->ju = (c->jitter[0] * 2.0f) / (float)c->width;
    q->jv = (c->jitter[1] * 2.0f) / (float)c->height;
}

/* Direction through the (jittered) centre of pixel (x, y) of a w x h grid. */
static void pixel_dir(const orc_camera *c, const lensq *q, int x, int y, int w, int h, float fv[3])
{
    float u = (((((float)x + 0.5f) * 2.0f) / (float)w - 1.0f) + q->ju) * q->tanx;
    float v = ((1.0f - (((float)y + 0.5f) * 2.0f) / (float)h) - q->jv) * q->tany;
    for (int a = 0; a < 3; a++) fv[a] = (c->fwd[a] + u * c->right[a]) + v * c->up[a];
}

static float view_depth(const orc_camera *c, const float p[3])
{
    return ((p[0] - c->pos[0]) * c->fwd[0] + (p[1] - c->pos[1]) * c->fwd[1]) + (p[2] - c->pos[2]) * c->fwd[2];
}

/* Support stage: all-in-focus G-buffer through the lens centre (the sharp
 * rasterized image of section 3), one sample per full-res pixel. */
int orc_gbuffer(const orc_scene *s, const orc_bvh *b, const orc_camera *cam,
                const orc_lens *lens, float *colour, float *depth, float *normal)
{
    if (!s || !cam || !lens || cam->width <= 0 || cam->height <= 0) return -1;
    int W = cam->width, H = cam->height;
    lensq q = lens_quantities(lens, W, H);
    set_jitter(&q, cam);
#pragma omp parallel for schedule(dynamic, 4) num_threads(g_threads)
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            size_t p = (size_t)y * W + x;
            float fv[3], d[3];
            pixel_dir(cam, &q, x, y, W, H, fv);
            float len = sqrtf((fv[0] * fv[0] + fv[1] * fv[1]) + fv[2] * fv[2]);
            for (int a = 0; a < 3; a++) d[a] = fv[a] / len;
            int32_t id;
            float t;
            closest(s, b, cam->pos, d, &id, &t);
            if (id >= 0) {
                float P[3], rgb[3], n[3];
                for (int a = 0; a < 3; a++) P[a] = cam->pos[a] + t * d[a];
                shade(s, (uint32_t)id, d, rgb, n);
                colour[4 * p + 0] = rgb[0]; colour[4 * p + 1] = rgb[1]; colour[4 * p + 2] = rgb[2];
                colour[4 * p + 3] = 1.0f;
                depth[p] = view_depth(cam, P);
                normal[4 * p + 0] = n[0]; normal[4 * p + 1] = n[1]; normal[4 * p + 2] = n[2];
                normal[4 * p + 3] = 0.0f;
            } else {
                colour[4 * p + 0] = s->sky[0]; colour[4 * p + 1] = s->sky[1]; colour[4 * p + 2] = s->sky[2];
                colour[4 * p + 3] = 1.0f;
                depth[p] = INFINITY;
                normal[4 * p + 0] = 0.0f; normal[4 * p + 1] = 0.0f; normal[4 * p + 2] = 0.0f;
                normal[4 * p + 3] = 0.0f;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Image helpers (clamp-to-edge everywhere)                                  */
/* ------------------------------------------------------------------------ */

/* Bilinear sample of a 4-channel image at continuous coordinates whose
 * integer values are texel centres. */
static void bilinear4(const float *img, int w, int h, float x, float y, float out[4])
{
    float x0f = floorf(x), y0f = floorf(y);
    float fx = x - x0f, fy = y - y0f;
    int x0 = (int)x0f, y0 = (int)y0f;
    int x1 = clampi(x0 + 1, 0, w - 1), y1 = clampi(y0 + 1, 0, h - 1);
    x0 = clampi(x0, 0, w - 1);
    y0 = clampi(y0, 0, h - 1);
    const float *a = img + 4 * ((size_t)y0 * w + x0), *b = img + 4 * ((size_t)y0 * w + x1);
    const float *c = img + 4 * ((size_t)y1 * w + x0), *d = img + 4 * ((size_t)y1 * w + x1);
    for (int k = 0; k < 4; k++) {
        float top = a[k] + (b[k] - a[k]) * fx;
        float bot = c[k] + (d[k] - c[k]) * fx;
        out[k] = top + (bot - top) * fy;
    }
}

static int nearest_index(float s, int n)
{
    return clampi((int)floorf(s + 0.5f), 0, n - 1);
}

static float median9(float *v)
{
    for (int i = 1; i < 9; i++) {
        float x = v[i];
        int j = i - 1;
        while (j >= 0 && v[j] > x) { v[j + 1] = v[j]; j--; }
        v[j + 1] = x;
    }
    return v[4];
}

/* 81-tap kernel of 3.1.1: the centre and four rings of 8k taps at radius k/4
 * of the kernel size, evenly spaced in angle (one more ring than the 49-tap
 * 3-ring kernel it extends). */
typedef struct {
    float ox[81], oy[81], frac[81];
} ring_table;

static ring_table make_rings(void)
{
    ring_table t;
    const double pi = 3.14159265358979323846;
    int i = 0;
    t.ox[0] = 0.0f; t.oy[0] = 0.0f; t.frac[0] = 0.0f;
    i = 1;
    for (int k = 1; k <= 4; k++) {
        for (int j = 0; j < 8 * k; j++, i++) {
            double th = 2.0 * pi * (double)j / (double)(8 * k);
            t.ox[i] = (float)(k / 4.0 * cos(th));
            t.oy[i] = (float)(k / 4.0 * sin(th));
            t.frac[i] = (float)k * 0.25f;
        }
    }
    return t;
}

/* The gather kernel shaped like the aperture (section 2 names polygonal
 * bokeh as an extension obtained by changing the shape of the sampling
 * kernel): ring k holds 8k taps at equal arc length on the aperture polygon
 * of circumradius k/4 (vertices at rot + 2 pi i / B, the corners between
 * the blade normals), the first half a step past vertex 0; a tap's distance
 * is k/4, its radius in the polygon's own norm.  Offsets take the far-field
 * image of the aperture on screen (lens up is screen -y), reflected for
 * gathering, i.e. lens point (x, y) becomes tap offset (-x, y). */
static ring_table make_polygon_rings(int blades, float rot)
{
    ring_table t;
    const double pi = 3.14159265358979323846;
    const double side = 2.0 * sin(pi / blades);
    t.ox[0] = 0.0f; t.oy[0] = 0.0f; t.frac[0] = 0.0f;
    int i = 1;
    for (int k = 1; k <= 4; k++) {
        const int n = 8 * k;
        for (int j = 0; j < n; j++, i++) {
            double s = ((double)j + 0.5) * ((double)blades * side) / (double)n;
            int e = (int)floor(s / side);
            if (e >= blades) e = blades - 1;
            double u = s / side - (double)e;
            double a0 = (double)rot + 2.0 * pi * e / blades, a1 = (double)rot + 2.0 * pi * (e + 1) / blades;
            double px = (1.0 - u) * cos(a0) + u * cos(a1), py = (1.0 - u) * sin(a0) + u * sin(a1);
            t.ox[i] = (float)(k / 4.0 * -px);
            t.oy[i] = (float)(k / 4.0 * py);
            t.frac[i] = (float)k * 0.25f;
        }
    }
    return t;
}

/* The 81 taps of the post-process gather for a lens and parameters (for
 * tests): offsets in units of the kernel radius and ring distances. */
int orc_gather_rings(const orc_lens *lens, const orc_params *p, float *ox, float *oy, float *frac)
{
    if (!lens || !p || !ox || !oy || !frac) return -1;
    ring_table t = (p->pp_polygon && lens->blades >= 3) ? make_polygon_rings(lens->blades, lens->blade_rot)
                                                       : make_rings();
    memcpy(ox, t.ox, sizeof(t.ox));
    memcpy(oy, t.oy, sizeof(t.oy));
    memcpy(frac, t.frac, sizeof(t.frac));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reprojection into the previous camera (3.2.3)                            */
/* ------------------------------------------------------------------------ */

/* Half-res texel of the previous frame that sees point p (or, when is_dir,
 * the point at infinity in direction p); -1 when behind or off screen. */
static int32_t reproject(const orc_camera *pc, const lensq *pq, int hw, int hh,
                         const float p[3], int is_dir)
{
    float e[3];
    for (int a = 0; a < 3; a++) e[a] = is_dir ? p[a] : p[a] - pc->pos[a];
    float ex = (e[0] * pc->right[0] + e[1] * pc->right[1]) + e[2] * pc->right[2];
    float ey = (e[0] * pc->up[0] + e[1] * pc->up[1]) + e[2] * pc->up[2];
    float ez = (e[0] * pc->fwd[0] + e[1] * pc->fwd[1]) + e[2] * pc->fwd[2];
    if (!(ez > 0.0f)) return -1;
    float pu = (ex / ez) / pq->tanx;
    float pv = (ey / ez) / pq->tany;
    float px = ((pu + 1.0f) * 0.5f) * (float)hw - 0.5f;
    float py = ((1.0f - pv) * 0.5f) * (float)hh - 0.5f;
    float sx = px + 0.5f, sy = py + 0.5f;
    if (!(sx >= 0.0f && sx < (float)hw && sy >= 0.0f && sy < (float)hh)) return -1;
    int ix = (int)floorf(sx), iy = (int)floorf(sy);
    return (int32_t)iy * hw + ix;
}

/* History record per half-res pixel: four planes.
 *   A (float4): accumulated near colour rgb, accumulated hit ratio
 *   B (float4): accumulated far colour rgb, age in frames
 *   C (float4): accumulated near CoC, far CoC, luma mean, luma second moment
 *   D (float) : blurred luminance variance */
#define HA(h, n, i) ((h) + 4 * (size_t)(i))
#define HB(h, n, i) ((h) + 4 * (size_t)(n) + 4 * (size_t)(i))
#define HC(h, n, i) ((h) + 8 * (size_t)(n) + 4 * (size_t)(i))
#define HD(h, n, i) ((h) + 12 * (size_t)(n) + (size_t)(i))

static int same_view(const orc_camera *a, const orc_camera *b, const orc_lens *la, const orc_lens *lb)
{
    return memcmp(a->pos, b->pos, sizeof(a->pos)) == 0 && memcmp(a->right, b->right, sizeof(a->right)) == 0 &&
           memcmp(a->up, b->up, sizeof(a->up)) == 0 && memcmp(a->fwd, b->fwd, sizeof(a->fwd)) == 0 &&
           memcmp(la, lb, sizeof(*la)) == 0;
}

/* ------------------------------------------------------------------------ */
/* The per-frame pass                                                        */
/* ------------------------------------------------------------------------ */

/* One TAA resolve (3.4, after Karis 2014) of the w x h float4 image `cur`,
 * whose pixel i sees view depth depth[i * dstride] through the jittered
 * camera: its colour is blended with the history image `hin` (the same grid;
 * NULL: none) fetched bilinearly where the pixel's point -- its direction for
 * the sky -- lands in the previous camera (none behind it or off the grid),
 * that history clamped per RGB channel to cur's range over the 3 x 3
 * neighbourhood (clamp to edge); history weight 0.9.  The result goes to out
 * and hout, its 4th channel 1, or cur's with keep_w. */
static void taa_resolve(const float *cur, const float *depth, int dstride, int w, int h, const orc_camera *cam,
                        const lensq *q, const orc_camera *pc, const lensq *pq, const float *hin, float *out,
                        float *hout, int keep_w)
{
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            size_t pidx = (size_t)y * w + x;
            float mn[3], mx[3];
            for (int cc = 0; cc < 3; cc++) { mn[cc] = INFINITY; mx[cc] = -INFINITY; }
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    const float *v = cur + 4 * ((size_t)clampi(y + dy, 0, h - 1) * w + clampi(x + dx, 0, w - 1));
                    for (int cc = 0; cc < 3; cc++) {
                        mn[cc] = v[cc] < mn[cc] ? v[cc] : mn[cc];
                        mx[cc] = v[cc] > mx[cc] ? v[cc] : mx[cc];
                    }
                }
            const float *c = cur + 4 * pidx;
            int valid = 0;
            float hcol[4];
            if (hin) {
                float fv[3], P[3], e[3];
                pixel_dir(cam, q, x, y, w, h, fv);
                float z = depth[pidx * (size_t)dstride];
                int isdir = !(z < INFINITY);
                for (int a = 0; a < 3; a++) P[a] = isdir ? fv[a] : cam->pos[a] + z * fv[a];
                for (int a = 0; a < 3; a++) e[a] = isdir ? P[a] : P[a] - pc->pos[a];
                float ex = (e[0] * pc->right[0] + e[1] * pc->right[1]) + e[2] * pc->right[2];
                float ey = (e[0] * pc->up[0] + e[1] * pc->up[1]) + e[2] * pc->up[2];
                float ez = (e[0] * pc->fwd[0] + e[1] * pc->fwd[1]) + e[2] * pc->fwd[2];
                if (ez > 0.0f) {
                    float pu = (ex / ez) / pq->tanx, pv = (ey / ez) / pq->tany;
                    float px = ((pu + 1.0f) * 0.5f) * (float)w - 0.5f;
                    float py = ((1.0f - pv) * 0.5f) * (float)h - 0.5f;
                    if (px + 0.5f >= 0.0f && px + 0.5f < (float)w && py + 0.5f >= 0.0f && py + 0.5f < (float)h) {
                        bilinear4(hin, w, h, px, py, hcol);
                        valid = 1;
                    }
                }
            }
            float o[4];
            for (int cc = 0; cc < 3; cc++) {
                float v = c[cc];
                if (valid) {
                    float hv = hcol[cc];
                    hv = hv > mn[cc] ? hv : mn[cc];
                    hv = hv < mx[cc] ? hv : mx[cc];
                    v = lerpf(c[cc], hv, 0.9f);
                }
                o[cc] = v;
            }
            o[3] = keep_w ? c[3] : 1.0f;
            for (int cc = 0; cc < 4; cc++) {
                out[4 * pidx + cc] = o[cc];
                hout[4 * pidx + cc] = o[cc];
            }
        }
}

int orc_render_frame(const orc_scene *s, const orc_bvh *b,
                     const orc_camera *cam, const orc_lens *lens,
                     const orc_camera *prev_cam, const orc_lens *prev_lens,
                     int32_t reset, const orc_params *p,
                     const float *gb_colour, const float *gb_depth,
                     const float *gb_normal, const float *hist_in,
                     float *hist_out, float *out_colour, uint8_t *out_mask,
                     orc_debug *dbg)
{
    if (!s || !cam || !lens || !p || !gb_colour || !gb_depth || !gb_normal || !hist_out || !out_colour || !out_mask)
        return -1;
    const int W = cam->width, H = cam->height;
    if (W <= 0 || H <= 0 || (W & 1) || (H & 1)) return -1;
    if (p->m < 1 || p->m > 255 || p->tile < 1) return -1;
    if (lens->blades > 16 || (lens->blades > 0 && lens->blades < 3)) return -1;
    const int hw = W / 2, hh = H / 2;
    const size_t np = (size_t)hw * hh;
    const int T = p->tile, tw = (hw + T - 1) / T, th = (hh + T - 1) / T;
    const float d = lens->focus;
    lensq q = lens_quantities(lens, W, H);
    set_jitter(&q, cam);
    int have_hist = !reset && hist_in && prev_cam && prev_lens && prev_cam->width == W && prev_cam->height == H;
    int motion = have_hist ? !same_view(cam, prev_cam, lens, prev_lens) : 0;
    lensq pq = have_hist ? lens_quantities(prev_lens, W, H) : q;
    const ring_table rings = make_rings();
    /* the post-process gather's kernel: circles, or the aperture polygon */
    const ring_table grings = (p->pp_polygon && lens->blades >= 3) ? make_polygon_rings(lens->blades, lens->blade_rot)
                                                                   : rings;
    const aperture ap = make_aperture(lens->blades, lens->blade_rot);

    float *colr = (float *)calloc(np * 4, sizeof(float));
    float *zn = (float *)calloc(np * 4, sizeof(float));
    float *tmax = (float *)calloc((size_t)tw * th, sizeof(float));
    float *tdil = (float *)calloc((size_t)tw * th, sizeof(float));
    float *pre = (float *)calloc(np * 4, sizeof(float));
    float *gat = (float *)calloc(np * 4, sizeof(float));
    float *ppm = (float *)calloc(np * 4, sizeof(float));
    int32_t *prev = (int32_t *)calloc(np, sizeof(int32_t));
    uint32_t *queue = (uint32_t *)calloc(np, sizeof(uint32_t));
    uint32_t *rbase = (uint32_t *)calloc(np, sizeof(uint32_t));
    float *res = (float *)calloc(np * 16, sizeof(float));
    float *tmp = (float *)calloc(np * 8, sizeof(float));
    float *var = (float *)calloc(np, sizeof(float));
    float *vblur = (float *)calloc(np, sizeof(float));
    float *rtmed = (float *)calloc(np * 4, sizeof(float));
    float *rec = (float *)calloc(np * 4, sizeof(float));
    float *hblur = (float *)calloc(np * 4, sizeof(float));
    float *gblur = (float *)calloc(np * 4, sizeof(float));
    int mw[4], mh[4];
    size_t moff[4], mtot = 0;
    mw[0] = hw; mh[0] = hh;
    for (int L = 1; L < 4; L++) { mw[L] = (mw[L - 1] + 1) >> 1; mh[L] = (mh[L - 1] + 1) >> 1; }
    for (int L = 0; L < 4; L++) { moff[L] = mtot; mtot += (size_t)mw[L] * mh[L] * 4; }
    float *mips = (float *)calloc(mtot, sizeof(float));
    const int taa_final = (p->taa & ORC_TAA_FINAL) != 0, taa_rast = (p->taa & ORC_TAA_RASTER) != 0,
              taa_post = (p->taa & ORC_TAA_POST) != 0;
    float *rast = taa_rast ? (float *)calloc((size_t)W * H * 4, sizeof(float)) : NULL;
    float *ppt = taa_post ? (float *)calloc(np * 4, sizeof(float)) : NULL;
    float *comp = taa_final ? (float *)calloc((size_t)W * H * 4, sizeof(float)) : NULL;
    /* allocated later; every exit frees each buffer once (free(NULL) is a no-op) */
    int32_t *rhit = NULL;
    float *rt = NULL, *rcol = NULL, *rpos = NULL;
    int status = 0;
    if (!colr || !zn || !tmax || !tdil || !pre || !gat || !ppm || !prev || !queue || !rbase || !res || !tmp ||
        !var || !vblur || !rtmed || !rec || !hblur || !gblur || !mips || (taa_rast && !rast) || (taa_post && !ppt) ||
        (taa_final && !comp)) {
        status = -2;
        goto done;
    }

    /* History layout: the half-res record (13 floats per half-res pixel),
     * then from its size rounded up to 16 bytes three TAA planes of float4
     * per pixel: the final image's (full res), the raster image's (full res)
     * and the post-filter output's (half res). */
    const size_t taa_off = (13 * np + 3) & ~(size_t)3;
    const size_t rast_off = taa_off + 4 * (size_t)W * H, post_off = rast_off + 4 * (size_t)W * H;
    const float *hist_ok = have_hist ? hist_in : NULL;

    /* A0 -- TAA of the raster image before filtering (3.4), with
     * ORC_TAA_RASTER: every later stage reads the resolved colour. */
    const float *gbc = gb_colour;
    if (taa_rast) {
        taa_resolve(gb_colour, gb_depth, 1, W, H, cam, &q, prev_cam, &pq, hist_ok ? hist_ok + rast_off : NULL, rast,
                    hist_out + rast_off, 0);
        gbc = rast;
    }

    /* A1 -- CoC and half-resolution reduce (3.1: the image is downscaled to
     * half resolution; 3.3, eq. 6: the thin-lens CoC).  The quad keeps its
     * nearest texel (first in TL, TR, BL, BR order on ties) and its normal;
     * colour is the box average.  The signed radius is negative in the near
     * field (in front of the focus plane, section 3) and clamped to r_max. */
    for (int y = 0; y < hh; y++)
        for (int x = 0; x < hw; x++) {
            size_t t[4] = {(size_t)(2 * y) * W + 2 * x, (size_t)(2 * y) * W + 2 * x + 1,
                           (size_t)(2 * y + 1) * W + 2 * x, (size_t)(2 * y + 1) * W + 2 * x + 1};
            int sel = 0;
            float z = gb_depth[t[0]];
            for (int k = 1; k < 4; k++)
                if (gb_depth[t[k]] < z) { z = gb_depth[t[k]]; sel = k; }
            size_t i = (size_t)y * hw + x;
            for (int c = 0; c < 3; c++)
                colr[4 * i + c] = ((gbc[4 * t[0] + c] + gbc[4 * t[1] + c]) + (gbc[4 * t[2] + c] + gbc[4 * t[3] + c])) *
                                  0.25f;
            float r = coc_of(&q, d, z) * 0.25f;
            r = fmin_cs(r, p->r_max);
            colr[4 * i + 3] = z < d ? -r : r;
            zn[4 * i + 0] = z;
            for (int c = 0; c < 3; c++) zn[4 * i + 1 + c] = gb_normal[4 * t[sel] + c];
        }

    /* A2 -- maximum CoC per tile and over the tile neighbourhood (3.1.1). */
    const int D = (int)ceilf(p->r_max / (float)T);
    for (int ty = 0; ty < th; ty++)
        for (int tx = 0; tx < tw; tx++) {
            float m = 0.0f;
            for (int y = ty * T; y < (ty + 1) * T && y < hh; y++)
                for (int x = tx * T; x < (tx + 1) * T && x < hw; x++) m = fmax_cs(m, fabsf(colr[4 * ((size_t)y * hw + x) + 3]));
            tmax[(size_t)ty * tw + tx] = m;
        }
    for (int ty = 0; ty < th; ty++)
        for (int tx = 0; tx < tw; tx++) {
            float m = 0.0f;
            for (int j = ty - D; j <= ty + D; j++)
                for (int i = tx - D; i <= tx + D; i++)
                    if (i >= 0 && j >= 0 && i < tw && j < th) m = fmax_cs(m, tmax[(size_t)j * tw + i]);
            tdil[(size_t)ty * tw + tx] = m;
        }

    /* A3 -- 9-tap bilateral prefilter (3.1.1).  Kernel diameter 1/8 of the
     * neighbourhood maximum CoC diameter, never below sqrt(2); taps on a 3x3
     * grid; weight 1 / (1 + |r_i - r_c|).  Pinned at one CoC on a quadratic
     * field (tap spacing, sampling, normalisation) and across a step of the
     * CoC (the weight). */
    for (int y = 0; y < hh; y++)
        for (int x = 0; x < hw; x++) {
            size_t i = (size_t)y * hw + x;
            float Rn = tdil[(size_t)(y / T) * tw + x / T];
            float dpre = Rn * 0.25f;
            if (dpre < OR_SQRT2) dpre = OR_SQRT2;
            float sp = dpre * 0.5f;
            float rc = colr[4 * i + 3];
            float acc[3] = {0, 0, 0}, sw = 0.0f;
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    float sx = (float)x + (float)dx * sp, sy = (float)y + (float)dy * sp;
                    float v[4];
                    bilinear4(colr, hw, hh, sx, sy, v);
                    float w = 1.0f / (1.0f + fabsf(v[3] - rc));
                    for (int c = 0; c < 3; c++) acc[c] = acc[c] + w * v[c];
                    sw = sw + w;
                }
            for (int c = 0; c < 3; c++) pre[4 * i + c] = acc[c] / sw;
            pre[4 * i + 3] = rc;
        }

    /* A4 -- 81-tap main filter, eq. (1) (3.1.2).  Tap i contributes when its
     * CoC radius exceeds its distance to the centre (D(0,i)); foreground and
     * background sums v_f, v_b are split by a depth ramp over depth_range
     * (10 cm, 4.2); the undefined sampleAlpha is 1 / max(|r|, 1/2)^2; a
     * background tap also needs the centre's radius to reach it.  The
     * proportion of weight on taps brighter than l_spec is the bokeh
     * intensity used by the composite.  Pinned at one CoC and one depth
     * (inclusion, nearest-texel sampling, normalisation, bokeh share) and
     * across steps of depth and CoC (sampleAlpha, the foreground/background
     * split, the centre-radius rule for background taps). */
#pragma omp parallel for schedule(dynamic, 4) num_threads(g_threads)
    for (int y = 0; y < hh; y++)
        for (int x = 0; x < hw; x++) {
            size_t i = (size_t)y * hw + x;
            float Rn = tdil[(size_t)(y / T) * tw + x / T];
            float rc = pre[4 * i + 3], zc = zn[4 * i];
            float arc = fabsf(rc);
            float vf[3] = {0, 0, 0}, vb[3] = {0, 0, 0}, sw = 0.0f, ss = 0.0f;
            for (int k = 0; k < 81; k++) {
                float dist = Rn * grings.frac[k];
                float sx = (float)x + grings.ox[k] * Rn, sy = (float)y + grings.oy[k] * Rn;
                int ix = nearest_index(sx, hw), iy = nearest_index(sy, hh);
                size_t j = (size_t)iy * hw + ix;
                const float *ci = pre + 4 * j;
                float ari = fabsf(ci[3]);
                float mr = fmax_cs(ari, 0.5f);
                float alpha = 1.0f / (mr * mr);
                float dfg = ari > dist ? 1.0f : 0.0f;
                float dbg_ = fmin_cs(ari, arc) > dist ? 1.0f : 0.0f;
                float wbg = sat((zn[4 * j] - zc) / p->depth_range);
                float wf = alpha * ((1.0f - wbg) * dfg);
                float wb = alpha * (wbg * dbg_);
                for (int c = 0; c < 3; c++) {
                    vf[c] = vf[c] + wf * ci[c];
                    vb[c] = vb[c] + wb * ci[c];
                }
                float wi = wf + wb;
                sw = sw + wi;
                if (luma(ci[0], ci[1], ci[2]) > p->l_spec) ss = ss + wi;
            }
            if (sw > 0.0f) {
                for (int c = 0; c < 3; c++) gat[4 * i + c] = (vf[c] + vb[c]) / sw;
                gat[4 * i + 3] = ss / sw;
            } else {
                for (int c = 0; c < 3; c++) gat[4 * i + c] = pre[4 * i + c];
                gat[4 * i + 3] = 0.0f;
            }
        }

    /* A5 -- 3x3 median postfilter at half resolution (3.1.3); the upscale to
     * full resolution happens in the composite. */
    for (int y = 0; y < hh; y++)
        for (int x = 0; x < hw; x++) {
            size_t i = (size_t)y * hw + x;
            for (int c = 0; c < 3; c++) {
                float v[9];
                int n = 0;
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++)
                        v[n++] = gat[4 * ((size_t)clampi(y + dy, 0, hh - 1) * hw + clampi(x + dx, 0, hw - 1)) + c];
                ppm[4 * i + c] = median9(v);
            }
            ppm[4 * i + 3] = gat[4 * i + 3];
        }

    /* A5b -- TAA of the post-filter output (3.4), with ORC_TAA_POST, at half
     * resolution (the quad's nearest depth locates each pixel); the composite
     * reads the resolved image.  Its 4th channel passes through. */
    const float *ppc = ppm;
    if (taa_post) {
        taa_resolve(ppm, zn, 4, hw, hh, cam, &q, prev_cam, &pq, hist_ok ? hist_ok + post_off : NULL, ppt,
                    hist_out + post_off, 1);
        ppc = ppt;
    }

    /* A6 -- ray mask, eqs. (2)-(4) (3.2.1).  Gaussian (binomial 5-tap) on the
     * half-res depth feature d / z and the normals, then a 5x5 Sobel whose
     * gain is 1 per unit slope; x = (dd + dn) s, x_n = saturate(1 - 1/(x+1)), x_f = saturate(x_n
     * + var * 1e5) m; the count is x_f rounded to nearest, at least one ray for
     * an out-of-focus near-field pixel, never more than m.  The variance is
     * the previous frame's blurred estimate at the reprojected texel. */
    {
        static const float g5[5] = {0.0625f, 0.25f, 0.375f, 0.25f, 0.0625f};
        static const float sm[5] = {1.0f, 4.0f, 6.0f, 4.0f, 1.0f};
        static const float dv[5] = {-1.0f, -2.0f, 0.0f, 2.0f, 1.0f};
        /* channels: 0 = depth feature d / z (focus distance over view depth,
         * 0 for the sky), 1..3 = normal */
        for (int y = 0; y < hh; y++)
            for (int x = 0; x < hw; x++)
                for (int c = 0; c < 4; c++) {
                    float acc = 0.0f;
                    for (int j = 0; j < 5; j++) {
                        size_t k = (size_t)y * hw + clampi(x + j - 2, 0, hw - 1);
                        float v = zn[4 * k + c];
                        if (c == 0) v = d / v;
                        acc = acc + g5[j] * v;
                    }
                    hblur[4 * ((size_t)y * hw + x) + c] = acc;
                }
        for (int y = 0; y < hh; y++)
            for (int x = 0; x < hw; x++)
                for (int c = 0; c < 4; c++) {
                    float acc = 0.0f;
                    for (int i = 0; i < 5; i++)
                        acc = acc + g5[i] * hblur[4 * ((size_t)clampi(y + i - 2, 0, hh - 1) * hw + x) + c];
                    gblur[4 * ((size_t)y * hw + x) + c] = acc;
                }
        for (int y = 0; y < hh; y++)
            for (int x = 0; x < hw; x++) {
                size_t i = (size_t)y * hw + x;
                float gx[4], gy[4];
                for (int c = 0; c < 4; c++) {
                    float ax = 0.0f, ay = 0.0f;
                    for (int r = 0; r < 5; r++) {
                        size_t row = (size_t)clampi(y + r - 2, 0, hh - 1) * hw;
                        float hx = 0.0f, hs = 0.0f;
                        for (int k = 0; k < 5; k++) {
                            float v = gblur[4 * (row + clampi(x + k - 2, 0, hw - 1)) + c];
                            hx = hx + dv[k] * v;
                            hs = hs + sm[k] * v;
                        }
                        ax = ax + sm[r] * hx;
                        ay = ay + dv[r] * hs;
                    }
                    gx[c] = ax * 0.0078125f;
                    gy[c] = ay * 0.0078125f;
                }
                float dd = sqrtf(gx[0] * gx[0] + gy[0] * gy[0]);
                float an = 0.0f;
                for (int c = 1; c < 4; c++) an = an + (gx[c] * gx[c] + gy[c] * gy[c]);
                float dn = sqrtf(an);
                float xx = (dd + dn) * p->s;
                float xn = sat(1.0f - 1.0f / (xx + 1.0f));
                /* near reprojection of this pixel's G-buffer point */
                float z = zn[4 * i];
                int32_t pi = -1;
                if (have_hist) {
                    float fv[3], P[3];
                    pixel_dir(cam, &q, x, y, hw, hh, fv);
                    int isdir = !(z < INFINITY);
                    for (int a = 0; a < 3; a++) P[a] = isdir ? fv[a] : cam->pos[a] + z * fv[a];
                    pi = reproject(prev_cam, &pq, hw, hh, P, isdir);
                    if (pi >= 0 && !(HB(hist_in, np, pi)[3] > 0.0f)) pi = -1;
                }
                prev[i] = pi;
                float var_prev = pi >= 0 ? *HD(hist_in, np, pi) : 0.0f;
                float xf = sat(xn + var_prev * p->var_mask_w) * (float)p->m;
                int cnt = (int)floorf(xf + 0.5f);
                int near_oof = (z < d) && (coc_of(&q, d, z) > OR_SQRT2);
                int n = cnt > near_oof ? cnt : near_oof;
                if (n > p->m) n = p->m;
                if (p->mask_mode == 1) n = n > 0 ? p->m : 0;
                if (p->mask_mode == 2) n = p->m;
                out_mask[i] = (uint8_t)n;
            }
    }

    /* Mask mode 3, the remedy 5.3 proposes for tiling near the camera: the
     * ray mask grown by the maximum CoC of the neighbourhood.  Each pixel
     * takes the largest adaptive count within a square window whose radius
     * is its tile's dilated maximum CoC radius (A2), rounded up, clipped to
     * the image. */
    if (p->mask_mode == 3) {
        uint8_t *raw = (uint8_t *)malloc(np ? np : 1);
        if (!raw) {
            status = -2;
            goto done;
        }
        memcpy(raw, out_mask, np);
        for (int y = 0; y < hh; y++)
            for (int x = 0; x < hw; x++) {
                int R = (int)ceilf(tdil[(size_t)(y / T) * tw + x / T]);
                uint8_t best = 0;
                for (int yy = y - R; yy <= y + R; yy++) {
                    if (yy < 0 || yy >= hh) continue;
                    for (int xx = x - R; xx <= x + R; xx++) {
                        if (xx < 0 || xx >= hw) continue;
                        uint8_t v = raw[(size_t)yy * hw + xx];
                        best = v > best ? v : best;
                    }
                }
                out_mask[(size_t)y * hw + x] = best;
            }
        free(raw);
    }

    /* A7 -- ordered list of masked pixels and their first ray (the GPU
     * dispatches rays only for these pixels). */
    size_t P = 0, R = 0;
    for (size_t i = 0; i < np; i++)
        if (out_mask[i]) {
            queue[P] = (uint32_t)i;
            rbase[P] = (uint32_t)R;
            R += out_mask[i];
            P++;
        }

    /* A9/A10 -- thin-lens rays (3.2.2, after Cook 1984): from a random point
     * of the aperture towards the pixel's point on the focus plane at view
     * depth d, closest hit, Lambert shading.  Half resolution. */
    rhit = (int32_t *)malloc(sizeof(int32_t) * (R ? R : 1));
    rt = (float *)malloc(sizeof(float) * (R ? R : 1));
    rcol = (float *)malloc(sizeof(float) * 4 * (R ? R : 1));
    rpos = (float *)malloc(sizeof(float) * 4 * (R ? R : 1));
    if (!rhit || !rt || !rcol || !rpos) {
        status = -2;
        goto done;
    }
#pragma omp parallel for schedule(dynamic, 16) num_threads(g_threads)
    for (size_t j = 0; j < P; j++) {
        uint32_t qi = queue[j];
        int x = (int)(qi % (uint32_t)hw), y = (int)(qi / (uint32_t)hw);
        float fv[3], pf[3];
        pixel_dir(cam, &q, x, y, hw, hh, fv);
        for (int a = 0; a < 3; a++) pf[a] = cam->pos[a] + fv[a] * d;
        for (uint32_t k = 0; k < out_mask[qi]; k++) {
            size_t r = rbase[j] + k;
            float lx, ly, o[3], dir[3];
            lens_point(&ap, cam->seed, cam->frame, qi, k, &lx, &ly);
            for (int a = 0; a < 3; a++) o[a] = cam->pos[a] + q.half_a * (lx * cam->right[a] + ly * cam->up[a]);
            for (int a = 0; a < 3; a++) dir[a] = pf[a] - o[a];
            float len = sqrtf((dir[0] * dir[0] + dir[1] * dir[1]) + dir[2] * dir[2]);
            for (int a = 0; a < 3; a++) dir[a] = dir[a] / len;
            int32_t id;
            float t;
            closest(s, b, o, dir, &id, &t);
            rhit[r] = id;
            rt[r] = t;
            if (id >= 0) {
                float Ph[3], rgb[3];
                for (int a = 0; a < 3; a++) Ph[a] = o[a] + t * dir[a];
                shade(s, (uint32_t)id, dir, rgb, NULL);
                rcol[4 * r + 0] = rgb[0]; rcol[4 * r + 1] = rgb[1]; rcol[4 * r + 2] = rgb[2];
                rcol[4 * r + 3] = view_depth(cam, Ph);
                rpos[4 * r + 0] = Ph[0]; rpos[4 * r + 1] = Ph[1]; rpos[4 * r + 2] = Ph[2];
            } else {
                rcol[4 * r + 0] = s->sky[0]; rcol[4 * r + 1] = s->sky[1]; rcol[4 * r + 2] = s->sky[2];
                rcol[4 * r + 3] = INFINITY;
                rpos[4 * r + 0] = 0.0f; rpos[4 * r + 1] = 0.0f; rpos[4 * r + 2] = 0.0f;
            }
            rpos[4 * r + 3] = 0.0f;
        }
    }

    /* A11 -- split each pixel's rays into near and far field by distance from
     * the focus plane with a linear ramp (3.2.2), hit ratio = near weight /
     * rays shot, per-field mean colour and CoC, mean far-field hit position
     * (3.2.3).  Planes: R0 near rgb + N, R1 far rgb + h, R2 cN, cF, n, 0,
     * R3 far position + validity. */
    float *R0 = res, *R1 = res + 4 * np, *R2 = res + 8 * np, *R3 = res + 12 * np;
    for (size_t j = 0; j < P; j++) {
        uint32_t qi = queue[j];
        int n = out_mask[qi];
        float N = 0.0f, sn[3] = {0, 0, 0}, sf[3] = {0, 0, 0}, scn = 0.0f, scf = 0.0f;
        float fp[3] = {0, 0, 0}, fw = 0.0f;
        for (int k = 0; k < n; k++) {
            size_t r = rbase[j] + k;
            float z = rcol[4 * r + 3];
            int hit = rhit[r] >= 0;
            float w = hit ? sat(0.5f + (d - z) / q.ramp) : 0.0f;
            float om = 1.0f - w;
            float cz = coc_of(&q, d, z);
            N = N + w;
            for (int c = 0; c < 3; c++) {
                sn[c] = sn[c] + w * rcol[4 * r + c];
                sf[c] = sf[c] + om * rcol[4 * r + c];
            }
            scn = scn + w * cz;
            scf = scf + om * cz;
            if (hit) {
                for (int a = 0; a < 3; a++) fp[a] = fp[a] + om * rpos[4 * r + a];
                fw = fw + om;
            }
        }
        float nf = (float)n - N;
        for (int c = 0; c < 3; c++) {
            R0[4 * qi + c] = N > 0.0f ? sn[c] / N : 0.0f;
            R1[4 * qi + c] = nf > 0.0f ? sf[c] / nf : 0.0f;
        }
        R0[4 * qi + 3] = N;
        R1[4 * qi + 3] = N / (float)n;
        R2[4 * qi + 0] = N > 0.0f ? scn / N : 0.0f;
        R2[4 * qi + 1] = nf > 0.0f ? scf / nf : 0.0f;
        R2[4 * qi + 2] = (float)n;
        R2[4 * qi + 3] = 0.0f;
        for (int a = 0; a < 3; a++) R3[4 * qi + a] = fw > 0.0f ? fp[a] / fw : 0.0f;
        R3[4 * qi + 3] = fw > 0.0f ? 1.0f : 0.0f;
    }

    /* A12 -- temporal accumulation and reprojection (3.2.3).  Exponential
     * moving average with history weight alpha (0.95; reduced during
     * motion), near field reprojected with the G-buffer point, far field with
     * the mean far hit position (else the mean of valid 3x3 neighbours),
     * colour and CoC merged by the hit ratio (the latest one during motion),
     * luminance moments give the variance (after SVGF).  Planes: T0 c_rt rgb
     * + validity, T1 c_t, h_use, variance, 0. */
    float *T0 = tmp, *T1 = tmp + 4 * np;
    const float ah = motion ? p->alpha_motion : p->alpha;
    for (int y = 0; y < hh; y++)
        for (int x = 0; x < hw; x++) {
            size_t i = (size_t)y * hw + x;
            float *ha = HA(hist_out, np, i), *hb = HB(hist_out, np, i), *hc = HC(hist_out, np, i);
            int n = out_mask[i];
            if (n == 0) {
                for (int c = 0; c < 4; c++) { T0[4 * i + c] = 0.0f; T1[4 * i + c] = 0.0f; ha[c] = 0.0f; hb[c] = 0.0f; hc[c] = 0.0f; }
                var[i] = 0.0f;
                continue;
            }
            float N = R0[4 * i + 3], hcur = R1[4 * i + 3];
            float nf = (float)n - N;
            int32_t pn = prev[i];
            int vn = pn >= 0;
            /* far position: own, else mean of valid 3x3 neighbours */
            float fpos[3];
            int fvalid = R3[4 * i + 3] > 0.0f;
            if (fvalid) {
                for (int a = 0; a < 3; a++) fpos[a] = R3[4 * i + a];
            } else {
                float acc[3] = {0, 0, 0};
                int cnt = 0;
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        int xx = x + dx, yy = y + dy;
                        if ((dx == 0 && dy == 0) || xx < 0 || yy < 0 || xx >= hw || yy >= hh) continue;
                        size_t k = (size_t)yy * hw + xx;
                        if (out_mask[k] && R3[4 * k + 3] > 0.0f) {
                            for (int a = 0; a < 3; a++) acc[a] = acc[a] + R3[4 * k + a];
                            cnt++;
                        }
                    }
                if (cnt > 0) {
                    for (int a = 0; a < 3; a++) fpos[a] = acc[a] / (float)cnt;
                    fvalid = 1;
                }
            }
            int32_t pf_ = -1;
            if (have_hist && fvalid) {
                pf_ = reproject(prev_cam, &pq, hw, hh, fpos, 0);
                if (pf_ >= 0 && !(HB(hist_in, np, pf_)[3] > 0.0f)) pf_ = -1;
            }
            int vf = pf_ >= 0;
            const float *hNa = vn ? HA(hist_in, np, pn) : NULL, *hNb = vn ? HB(hist_in, np, pn) : NULL;
            const float *hNc = vn ? HC(hist_in, np, pn) : NULL;
            const float *hFb = vf ? HB(hist_in, np, pf_) : NULL, *hFc = vf ? HC(hist_in, np, pf_) : NULL;
            float accN[3], accF[3];
            for (int c = 0; c < 3; c++) {
                float cur = R0[4 * i + c];
                accN[c] = N > 0.0f ? (vn ? lerpf(cur, hNa[c], ah) : cur) : (vn ? hNa[c] : 0.0f);
                float cf = R1[4 * i + c];
                accF[c] = nf > 0.0f ? (vf ? lerpf(cf, hFb[c], ah) : cf) : (vf ? hFb[c] : 0.0f);
            }
            float cn = R2[4 * i + 0], cfv = R2[4 * i + 1];
            float accCN = N > 0.0f ? (vn ? lerpf(cn, hNc[0], ah) : cn) : (vn ? hNc[0] : 0.0f);
            float accCF = nf > 0.0f ? (vf ? lerpf(cfv, hFc[1], ah) : cfv) : (vf ? hFc[1] : 0.0f);
            float accH = vn ? lerpf(hcur, hNa[3], ah) : hcur;
            float huse = motion ? hcur : accH;
            float crt[3];
            for (int c = 0; c < 3; c++) crt[c] = lerpf(accF[c], accN[c], huse);
            float ct = lerpf(accCF, accCN, huse);
            float l = luma(crt[0], crt[1], crt[2]);
            float mu1 = vn ? lerpf(l, hNc[2], ah) : l;
            float mu2 = vn ? lerpf(l * l, hNc[3], ah) : l * l;
            float v = mu2 - mu1 * mu1;
            v = v > 0.0f ? v : 0.0f;
            float age = vn ? hNb[3] + 1.0f : 1.0f;
            for (int c = 0; c < 3; c++) { T0[4 * i + c] = crt[c]; ha[c] = accN[c]; hb[c] = accF[c]; }
            T0[4 * i + 3] = 1.0f;
            T1[4 * i + 0] = ct; T1[4 * i + 1] = huse; T1[4 * i + 2] = v; T1[4 * i + 3] = 0.0f;
            ha[3] = accH;
            hb[3] = age;
            hc[0] = accCN; hc[1] = accCF; hc[2] = mu1; hc[3] = mu2;
            var[i] = v;
        }
    /* Gaussian (3x3 binomial) blur of the variance (3.2.3). */
    {
        static const float g3[3] = {0.25f, 0.5f, 0.25f};
        for (int y = 0; y < hh; y++)
            for (int x = 0; x < hw; x++) {
                float acc = 0.0f;
                for (int r = 0; r < 3; r++) {
                    size_t row = (size_t)clampi(y + r - 1, 0, hh - 1) * hw;
                    float hs = 0.0f;
                    for (int k = 0; k < 3; k++) hs = hs + g3[k] * var[row + clampi(x + k - 1, 0, hw - 1)];
                    acc = acc + g3[r] * hs;
                }
                size_t i = (size_t)y * hw + x;
                vblur[i] = acc;
                *HD(hist_out, np, i) = acc;
            }
    }

    /* A13 -- median of the ray-traced colour, then spatial reconstruction
     * (3.2.4): circular 81-tap kernel scaled by the accumulated CoC, mip level
     * from eq. (8), taps whose CoC radius is below their distance rejected,
     * neighbourhood mean blended in by b of eq. (5).  Invalid neighbours are
     * replaced by the centre in the median and carry zero weight in the
     * validity-weighted mip chain. */
    for (int y = 0; y < hh; y++)
        for (int x = 0; x < hw; x++) {
            size_t i = (size_t)y * hw + x;
            if (!(T0[4 * i + 3] > 0.0f)) {
                for (int c = 0; c < 4; c++) rtmed[4 * i + c] = 0.0f;
                continue;
            }
            for (int c = 0; c < 3; c++) {
                float v[9];
                int n = 0;
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        size_t k = (size_t)clampi(y + dy, 0, hh - 1) * hw + clampi(x + dx, 0, hw - 1);
                        v[n++] = T0[4 * k + 3] > 0.0f ? T0[4 * k + c] : T0[4 * i + c];
                    }
                rtmed[4 * i + c] = median9(v);
            }
            rtmed[4 * i + 3] = 1.0f;
        }
    for (size_t i = 0; i < np; i++) {
        float v = rtmed[4 * i + 3];
        for (int c = 0; c < 3; c++) mips[moff[0] + 4 * i + c] = rtmed[4 * i + c] * v;
        mips[moff[0] + 4 * i + 3] = v;
    }
    for (int L = 1; L < 4; L++) {
        const float *src = mips + moff[L - 1];
        float *dst = mips + moff[L];
        int sw_ = mw[L - 1], sh_ = mh[L - 1];
        for (int y = 0; y < mh[L]; y++)
            for (int x = 0; x < mw[L]; x++) {
                int x0 = 2 * x, y0 = 2 * y, x1 = clampi(2 * x + 1, 0, sw_ - 1), y1 = clampi(2 * y + 1, 0, sh_ - 1);
                for (int c = 0; c < 4; c++) {
                    float a = src[4 * ((size_t)y0 * sw_ + x0) + c], bb = src[4 * ((size_t)y0 * sw_ + x1) + c];
                    float cc = src[4 * ((size_t)y1 * sw_ + x0) + c], dd = src[4 * ((size_t)y1 * sw_ + x1) + c];
                    dst[4 * ((size_t)y * mw[L] + x) + c] = ((a + bb) + (cc + dd)) * 0.25f;
                }
            }
    }
    for (int y = 0; y < hh; y++)
        for (int x = 0; x < hw; x++) {
            size_t i = (size_t)y * hw + x;
            if (!(T0[4 * i + 3] > 0.0f)) {
                for (int c = 0; c < 4; c++) rec[4 * i + c] = 0.0f;
                continue;
            }
            float ct = T1[4 * i + 0], hu = T1[4 * i + 1];
            float Rr = fmin_cs(ct * 0.25f, p->r_max);
            float lod = clampf(ct * p->lod_scale, 0.0f, p->lod_max);
            int L0 = (int)floorf(lod);
            int Lmax = (int)p->lod_max;
            if (Lmax > 3) Lmax = 3;
            if (L0 > Lmax) L0 = Lmax;
            int L1 = L0 < Lmax ? L0 + 1 : Lmax;
            float fl = lod - (float)L0;
            float acc[4] = {0, 0, 0, 0}, sh = 0.0f;
            int na = 0;
            for (int k = 0; k < 81; k++) {
                float dist = Rr * rings.frac[k];
                float sx = (float)x + rings.ox[k] * Rr, sy = (float)y + rings.oy[k] * Rr;
                int ix = nearest_index(sx, hw), iy = nearest_index(sy, hh);
                size_t j = (size_t)iy * hw + ix;
                if (!(T0[4 * j + 3] > 0.0f)) continue;
                if (T1[4 * j] * 0.25f < dist) continue;
                float s0[4], s1[4];
                float sc0 = 1.0f, sc1 = 1.0f;
                for (int L = 0; L < L0; L++) sc0 = sc0 * 0.5f;
                for (int L = 0; L < L1; L++) sc1 = sc1 * 0.5f;
                bilinear4(mips + moff[L0], mw[L0], mh[L0], (sx + 0.5f) * sc0 - 0.5f, (sy + 0.5f) * sc0 - 0.5f, s0);
                bilinear4(mips + moff[L1], mw[L1], mh[L1], (sx + 0.5f) * sc1 - 0.5f, (sy + 0.5f) * sc1 - 0.5f, s1);
                for (int c = 0; c < 4; c++) acc[c] = acc[c] + lerpf(s0[c], s1[c], fl);
                sh = sh + T1[4 * j + 1];
                na++;
            }
            float nb[3];
            for (int c = 0; c < 3; c++) nb[c] = acc[3] > 0.0f ? acc[c] / acc[3] : rtmed[4 * i + c];
            float hnb = na > 0 ? sh / (float)na : hu;
            float bb = clampf(vblur[i] * p->var_recon_w, 0.0f, p->b_max);
            for (int c = 0; c < 3; c++) rec[4 * i + c] = lerpf(rtmed[4 * i + c], nb[c], bb);
            rec[4 * i + 3] = lerpf(hu, hnb, bb);
        }

    /* A14 -- composite (3.3).  Inside the zone of focus (CoC <= sqrt(2),
     * eq. 6) the sharp raster colour, unless ray-traced foreground covers the
     * pixel; near field: ray-traced colour, pulled towards post-process by the
     * bokeh proportion; far field: blend by smoothstep(0, 0.3, h) of eq. (7),
     * weighting ray-traced colour where the hit ratio is at least 0.3. */
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            size_t pidx = (size_t)y * W + x;
            float z = gb_depth[pidx];
            float c = coc_of(&q, d, z);
            float hx = (float)x * 0.5f - 0.25f, hy = (float)y * 0.5f - 0.25f;
            float pp[4];
            bilinear4(ppc, hw, hh, hx, hy, pp);
            float x0f = floorf(hx), y0f = floorf(hy);
            float fx = hx - x0f, fy = hy - y0f;
            int x0 = (int)x0f, y0 = (int)y0f;
            int xs[2] = {clampi(x0, 0, hw - 1), clampi(x0 + 1, 0, hw - 1)};
            int ys[2] = {clampi(y0, 0, hh - 1), clampi(y0 + 1, 0, hh - 1)};
            float wts[4] = {(1.0f - fx) * (1.0f - fy), fx * (1.0f - fy), (1.0f - fx) * fy, fx * fy};
            float sw = 0.0f, rc[3] = {0, 0, 0}, rh = 0.0f, rct = 0.0f;
            for (int k = 0; k < 4; k++) {
                size_t j = (size_t)ys[k >> 1] * hw + xs[k & 1];
                float wv = wts[k] * T0[4 * j + 3];
                sw = sw + wv;
                for (int cc = 0; cc < 3; cc++) rc[cc] = rc[cc] + wv * rec[4 * j + cc];
                rh = rh + wv * rec[4 * j + 3];
                rct = rct + wv * T1[4 * j + 0];
            }
            int rtv = sw > 0.0f;
            if (rtv) {
                for (int cc = 0; cc < 3; cc++) rc[cc] = rc[cc] / sw;
                rh = rh / sw;
                rct = rct / sw;
            }
            float *o = out_colour + 4 * pidx;
            if (c <= OR_SQRT2 && (!rtv || rct < OR_SQRT2)) {
                for (int cc = 0; cc < 3; cc++) o[cc] = gbc[4 * pidx + cc];
            } else if (!rtv) {
                for (int cc = 0; cc < 3; cc++) o[cc] = pp[cc];
            } else if (z < d) {
                for (int cc = 0; cc < 3; cc++) o[cc] = lerpf(rc[cc], pp[cc], pp[3]);
            } else {
                float t = sat(rh / p->h_edge);
                float w = (t * t) * (3.0f - 2.0f * t);
                if (p->composite_literal) /* the literal reading of 3.3: high hit ratio -> post-process */
                    for (int cc = 0; cc < 3; cc++) o[cc] = lerpf(rc[cc], pp[cc], w);
                else
                    for (int cc = 0; cc < 3; cc++) o[cc] = lerpf(pp[cc], rc[cc], w);
            }
            o[3] = 1.0f;
        }

    /* A15 -- final temporal anti-aliasing (3.4, after Karis 2014), with
     * ORC_TAA_FINAL: the composite resolved against the previous output. */
    if (taa_final) {
        memcpy(comp, out_colour, sizeof(float) * 4 * (size_t)W * H);
        taa_resolve(comp, gb_depth, 1, W, H, cam, &q, prev_cam, &pq, hist_ok ? hist_ok + taa_off : NULL, out_colour,
                    hist_out + taa_off, 0);
    }

    if (dbg) {
        if (dbg->colr) memcpy(dbg->colr, colr, np * 16);
        if (dbg->zn) memcpy(dbg->zn, zn, np * 16);
        if (dbg->tile_max) memcpy(dbg->tile_max, tmax, (size_t)tw * th * 4);
        if (dbg->tile_dil) memcpy(dbg->tile_dil, tdil, (size_t)tw * th * 4);
        if (dbg->pre) memcpy(dbg->pre, pre, np * 16);
        if (dbg->gather) memcpy(dbg->gather, gat, np * 16);
        if (dbg->ppmed) memcpy(dbg->ppmed, ppm, np * 16);
        if (dbg->prev_idx) memcpy(dbg->prev_idx, prev, np * 4);
        if (dbg->queue) memcpy(dbg->queue, queue, P * 4);
        if (dbg->ray_base) memcpy(dbg->ray_base, rbase, P * 4);
        if (dbg->ray_hit) memcpy(dbg->ray_hit, rhit, R * 4);
        if (dbg->ray_t) memcpy(dbg->ray_t, rt, R * 4);
        if (dbg->ray_col) memcpy(dbg->ray_col, rcol, R * 16);
        if (dbg->ray_pos) memcpy(dbg->ray_pos, rpos, R * 16);
        if (dbg->resolve) memcpy(dbg->resolve, res, np * 64);
        if (dbg->temporal) memcpy(dbg->temporal, tmp, np * 32);
        if (dbg->var_blur) memcpy(dbg->var_blur, vblur, np * 4);
        if (dbg->rtmed) memcpy(dbg->rtmed, rtmed, np * 16);
        if (dbg->mips) memcpy(dbg->mips, mips, mtot * 4);
        if (dbg->recon) memcpy(dbg->recon, rec, np * 16);
        dbg->n_masked = (int64_t)P;
        dbg->n_rays = (int64_t)R;
    }
done:
    free(rhit); free(rt); free(rcol); free(rpos);
    free(colr); free(zn); free(tmax); free(tdil); free(pre); free(gat); free(ppm); free(prev);
    free(queue); free(rbase); free(res); free(tmp); free(var); free(vblur); free(rtmed); free(rec);
    free(hblur); free(gblur); free(mips); free(rast); free(ppt); free(comp);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Estimator and its reference (Cook's distributed ray tracing, 3.2.2)       */
/* ------------------------------------------------------------------------ */

static void lens_ray_colour(const orc_scene *s, const orc_bvh *b, const orc_camera *cam,
                            const lensq *q, float d, const float pf[3], float lx, float ly, float rgb[3])
{
    float o[3], dir[3];
    for (int a = 0; a < 3; a++) o[a] = cam->pos[a] + q->half_a * (lx * cam->right[a] + ly * cam->up[a]);
    for (int a = 0; a < 3; a++) dir[a] = pf[a] - o[a];
    float len = sqrtf((dir[0] * dir[0] + dir[1] * dir[1]) + dir[2] * dir[2]);
    for (int a = 0; a < 3; a++) dir[a] = dir[a] / len;
    int32_t id;
    float t;
    (void)d;
    closest(s, b, o, dir, &id, &t);
    if (id >= 0) shade(s, (uint32_t)id, dir, rgb, NULL);
    else { rgb[0] = s->sky[0]; rgb[1] = s->sky[1]; rgb[2] = s->sky[2]; }
}

int orc_pixel_estimate(const orc_scene *s, const orc_bvh *b, const orc_camera *cam,
                       const orc_lens *lens, int64_t nq, const uint32_t *qlist, int32_t spp, float *rgb)
{
    if (!s || !cam || !lens || spp < 1 || nq < 0) return -1;
    int W = cam->width, H = cam->height, hw = W / 2, hh = H / 2;
    lensq q = lens_quantities(lens, W, H);
    set_jitter(&q, cam);
    aperture ap = make_aperture(lens->blades, lens->blade_rot);
#pragma omp parallel for schedule(dynamic, 4) num_threads(g_threads)
    for (int64_t j = 0; j < nq; j++) {
        uint32_t qi = qlist[j];
        int x = (int)(qi % (uint32_t)hw), y = (int)(qi / (uint32_t)hw);
        float fv[3], pf[3];
        pixel_dir(cam, &q, x, y, hw, hh, fv);
        for (int a = 0; a < 3; a++) pf[a] = cam->pos[a] + fv[a] * lens->focus;
        double acc[3] = {0, 0, 0};
        for (int k = 0; k < spp; k++) {
            float lx, ly, c[3];
            lens_point(&ap, cam->seed, cam->frame, qi, (uint32_t)k, &lx, &ly);
            lens_ray_colour(s, b, cam, &q, lens->focus, pf, lx, ly, c);
            for (int a = 0; a < 3; a++) acc[a] += c[a];
        }
        for (int a = 0; a < 3; a++) rgb[3 * j + a] = (float)(acc[a] / spp);
    }
    return 0;
}

int orc_lens_integral(const orc_scene *s, const orc_bvh *b, const orc_camera *cam,
                      const orc_lens *lens, int64_t nq, const uint32_t *qlist, int32_t grid, float *rgb)
{
    if (!s || !cam || !lens || grid < 1 || nq < 0) return -1;
    int W = cam->width, H = cam->height, hw = W / 2, hh = H / 2;
    lensq q = lens_quantities(lens, W, H);
    set_jitter(&q, cam);
    aperture ap = make_aperture(lens->blades, lens->blade_rot);
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
    for (int64_t j = 0; j < nq; j++) {
        uint32_t qi = qlist[j];
        int x = (int)(qi % (uint32_t)hw), y = (int)(qi / (uint32_t)hw);
        float fv[3], pf[3];
        pixel_dir(cam, &q, x, y, hw, hh, fv);
        for (int a = 0; a < 3; a++) pf[a] = cam->pos[a] + fv[a] * lens->focus;
        double acc[3] = {0, 0, 0};
        long cnt = 0;
        for (int gy = 0; gy < grid; gy++)
            for (int gx = 0; gx < grid; gx++) {
                float lx = (float)((gx + 0.5) / grid * 2.0 - 1.0), ly = (float)((gy + 0.5) / grid * 2.0 - 1.0);
                if (!inside_aperture(&ap, lx, ly)) continue;
                float c[3];
                lens_ray_colour(s, b, cam, &q, lens->focus, pf, lx, ly, c);
                for (int a = 0; a < 3; a++) acc[a] += c[a];
                cnt++;
            }
        for (int a = 0; a < 3; a++) rgb[3 * j + a] = cnt ? (float)(acc[a] / cnt) : 0.0f;
    }
    return 0;
}
