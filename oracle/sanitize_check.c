/*
 * Memory and undefined-behaviour check of the CPU oracle (test
 * infrastructure).  Built by the test suite with AddressSanitizer,
 * LeakSanitizer and UndefinedBehaviorSanitizer, and with alloc_hook.h forced
 * into dof_oracle.c, it runs every entry point on a small scene -- each mask
 * mode, the TAA stages, a polygonal aperture, a second frame on the first
 * one's history, the estimator and its lens-grid reference, brute force and
 * BVH closest hits -- then repeats the allocating calls with each of their
 * allocations failing in turn and checks that they report -2.  A sanitizer
 * report or a wrong status ends the program with a nonzero exit code.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static long g_count = 0, g_fail_at = 0;

void *orc_hook_malloc(size_t n)
{
    long c = __atomic_add_fetch(&g_count, 1, __ATOMIC_SEQ_CST);
    return c == g_fail_at ? NULL : malloc(n);
}

void *orc_hook_calloc(size_t n, size_t size)
{
    long c = __atomic_add_fetch(&g_count, 1, __ATOMIC_SEQ_CST);
    return c == g_fail_at ? NULL : calloc(n, size);
}

static int g_errors = 0;
#define CHECK(cond)                                                         \
    do {                                                                    \
        if (!(cond)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            g_errors++;                                                     \
        }                                                                   \
    } while (0)

/* ---- a small scene: ground, boxes at 8-20, two thin bars near the camera */

static float g_verts[9 * 256], g_albedo[3 * 256];
static int g_ntri = 0;

static void tri(const float *a, const float *b, const float *c, float r, float g, float bl)
{
    memcpy(g_verts + 9 * g_ntri, a, 12);
    memcpy(g_verts + 9 * g_ntri + 3, b, 12);
    memcpy(g_verts + 9 * g_ntri + 6, c, 12);
    g_albedo[3 * g_ntri] = r;
    g_albedo[3 * g_ntri + 1] = g;
    g_albedo[3 * g_ntri + 2] = bl;
    g_ntri++;
}

static void quad(const float p[4][3], float r, float g, float b)
{
    tri(p[0], p[1], p[2], r, g, b);
    tri(p[0], p[2], p[3], r, g, b);
}

static void box(float x0, float y0, float z0, float x1, float y1, float z1, float r, float g, float b)
{
    const float f[6][4][3] = {
        {{x0, y0, z0}, {x0, y1, z0}, {x1, y1, z0}, {x1, y0, z0}}, {{x0, y0, z1}, {x1, y0, z1}, {x1, y1, z1}, {x0, y1, z1}},
        {{x0, y0, z0}, {x0, y0, z1}, {x0, y1, z1}, {x0, y1, z0}}, {{x1, y0, z0}, {x1, y1, z0}, {x1, y1, z1}, {x1, y0, z1}},
        {{x0, y0, z0}, {x1, y0, z0}, {x1, y0, z1}, {x0, y0, z1}}, {{x0, y1, z0}, {x0, y1, z1}, {x1, y1, z1}, {x1, y1, z0}},
    };
    for (int i = 0; i < 6; i++) quad(f[i], r, g, b);
}

static orc_scene make_scene(void)
{
    const float ground[4][3] = {{-60, 0, -1}, {-60, 0, 80}, {60, 0, 80}, {60, 0, -1}};
    quad(ground, 0.5f, 0.5f, 0.5f);
    box(-3, 0, 8, -1, 2, 9, 0.8f, 0.2f, 0.2f);
    box(1, 0, 12, 2.5f, 3, 13, 0.2f, 0.8f, 0.2f);
    box(-1, 0, 18, 1, 1.5f, 20, 0.2f, 0.2f, 0.8f);
    box(3, 0, 10, 4, 1, 11, 0.9f, 0.9f, 0.1f);
    box(-0.4f, 0, 1.8f, -0.38f, 3, 1.82f, 0.3f, 0.3f, 0.3f);
    box(0.5f, 0, 2.2f, 0.52f, 3, 2.22f, 0.6f, 0.4f, 0.2f);
    /* leaning grass blades: long thin triangles that the BVH splits into clipped pieces */
    for (int i = 0; i < 6; i++) {
        const float x = -1.5f + 0.5f * (float)i, z = 3.0f + 0.3f * (float)i;
        const float a[3] = {x, 0, z}, b[3] = {x + 0.02f, 0, z}, c[3] = {x + 0.3f, 1.2f, z + 0.2f};
        tri(a, b, c, 0.2f, 0.6f, 0.1f);
    }
    orc_scene s;
    memset(&s, 0, sizeof(s));
    s.ntri = g_ntri;
    s.verts = g_verts;
    s.albedo = g_albedo;
    s.leaf_split = 1;
    const float L[3] = {-0.4f, -1.0f, 0.6f};
    const float n = sqrtf(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
    for (int a = 0; a < 3; a++) {
        s.light_dir[a] = L[a] / n;
        s.light_rad[a] = 1.0f;
        s.ambient[a] = 0.15f;
    }
    s.sky[0] = 0.55f;
    s.sky[1] = 0.70f;
    s.sky[2] = 0.95f;
    return s;
}

static int alloc_bvh(orc_bvh *b, int n)
{
    memset(b, 0, sizeof(*b));
    b->nleaf = n;
    b->keys = malloc(sizeof(uint64_t) * n);
    b->refs = malloc(sizeof(uint32_t) * n);
    b->ids = malloc(sizeof(uint32_t) * n);
    b->left = malloc(sizeof(uint32_t) * (n - 1));
    b->right = malloc(sizeof(uint32_t) * (n - 1));
    b->parent = malloc(sizeof(uint32_t) * (2 * n - 1));
    b->bounds = malloc(sizeof(float) * 6 * (n - 1));
    b->leaf_bounds = malloc(sizeof(float) * 6 * n);
    return b->keys && b->refs && b->ids && b->left && b->right && b->parent && b->bounds && b->leaf_bounds;
}

static void free_bvh(orc_bvh *b)
{
    free(b->keys); free(b->refs); free(b->ids); free(b->left); free(b->right);
    free(b->parent); free(b->bounds); free(b->leaf_bounds);
}

static orc_camera camera(int W, int H, float x, uint32_t frame)
{
    orc_camera c;
    memset(&c, 0, sizeof(c));
    const float pos[3] = {x, 1.2f, 0.0f}, right[3] = {1, 0, 0}, up[3] = {0, 1, 0}, fwd[3] = {0, 0, 1};
    memcpy(c.pos, pos, 12);
    memcpy(c.right, right, 12);
    memcpy(c.up, up, 12);
    memcpy(c.fwd, fwd, 12);
    c.width = W;
    c.height = H;
    c.frame = frame;
    c.seed = 7;
    return c;
}

static orc_params params(int m, int mode, int taa, int polygon)
{
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.m = m;
    p.s = 0.8f;
    p.var_mask_w = 1e5f;
    p.alpha = 0.95f;
    p.alpha_motion = 0.8f;
    p.var_recon_w = 2000.0f;
    p.b_max = 0.9f;
    p.h_edge = 0.3f;
    p.lod_scale = 0.05f;
    p.lod_max = 3.0f;
    p.depth_range = 0.1f;
    p.r_max = 32.0f;
    p.tile = 16;
    p.l_spec = 1.0f;
    p.mask_mode = mode;
    p.pp_polygon = polygon;
    p.taa = taa;
    return p;
}

/* history floats of a W x H frame: the half-res record rounded to 16 bytes,
 * then the TAA planes (final and raster at full res, post-filter at half) */
static size_t hist_floats(int W, int H)
{
    size_t np = (size_t)(W / 2) * (H / 2);
    return ((13 * np + 3) & ~(size_t)3) + 8 * (size_t)W * H + 4 * np;
}

typedef struct {
    float *colour, *depth, *normal, *hist0, *hist1, *out;
    uint8_t *mask;
    orc_debug dbg;
    void *dbg_mem[20];
} frame_bufs;

static void bufs_alloc(frame_bufs *f, int W, int H, int m)
{
    const size_t np = (size_t)(W / 2) * (H / 2), nr = np * m, tiles = (size_t)((W / 2 + 15) / 16) * ((H / 2 + 15) / 16);
    f->colour = calloc((size_t)W * H * 4, sizeof(float));
    f->depth = calloc((size_t)W * H, sizeof(float));
    f->normal = calloc((size_t)W * H * 4, sizeof(float));
    f->hist0 = calloc(hist_floats(W, H), sizeof(float));
    f->hist1 = calloc(hist_floats(W, H), sizeof(float));
    f->out = calloc((size_t)W * H * 4, sizeof(float));
    f->mask = calloc(np, 1);
    const size_t sz[20] = {np * 16, np * 16, tiles * 4, tiles * 4, np * 16, np * 16, np * 16, np * 4, np * 4, np * 4,
                           nr * 4, nr * 4, nr * 16, nr * 16, np * 64, np * 32, np * 4, np * 16, np * 32, np * 16};
    for (int i = 0; i < 20; i++) f->dbg_mem[i] = calloc(sz[i], 1);
    memset(&f->dbg, 0, sizeof(f->dbg));
    void **slots[20] = {(void **)&f->dbg.colr, (void **)&f->dbg.zn, (void **)&f->dbg.tile_max, (void **)&f->dbg.tile_dil,
                        (void **)&f->dbg.pre, (void **)&f->dbg.gather, (void **)&f->dbg.ppmed, (void **)&f->dbg.prev_idx,
                        (void **)&f->dbg.queue, (void **)&f->dbg.ray_base, (void **)&f->dbg.ray_hit, (void **)&f->dbg.ray_t,
                        (void **)&f->dbg.ray_col, (void **)&f->dbg.ray_pos, (void **)&f->dbg.resolve,
                        (void **)&f->dbg.temporal, (void **)&f->dbg.var_blur, (void **)&f->dbg.rtmed,
                        (void **)&f->dbg.mips, (void **)&f->dbg.recon};
    for (int i = 0; i < 20; i++) *slots[i] = f->dbg_mem[i];
}

static void bufs_free(frame_bufs *f)
{
    free(f->colour); free(f->depth); free(f->normal); free(f->hist0); free(f->hist1); free(f->out); free(f->mask);
    for (int i = 0; i < 20; i++) free(f->dbg_mem[i]);
}

static int render(const orc_scene *s, const orc_bvh *b, frame_bufs *f, const orc_camera *c0, const orc_camera *c1,
                  const orc_lens *lens, const orc_params *p, int debug)
{
    int r = orc_render_frame(s, b, c0, lens, NULL, NULL, 1, p, f->colour, f->depth, f->normal, NULL, f->hist0, f->out,
                             f->mask, debug ? &f->dbg : NULL);
    if (r != 0) return r;
    return orc_render_frame(s, b, c1, lens, c0, lens, 0, p, f->colour, f->depth, f->normal, f->hist0, f->hist1,
                            f->out, f->mask, debug ? &f->dbg : NULL);
}

/* Runs call() once to count its allocations, then once per allocation with
 * that one failing; each failing run must return -2 (and free what it took). */
#define EACH_ALLOCATION_FAILS(call)                                                      \
    do {                                                                                 \
        g_fail_at = 0;                                                                   \
        g_count = 0;                                                                     \
        CHECK((call) == 0);                                                              \
        long n_ = g_count;                                                               \
        CHECK(n_ > 0);                                                                   \
        for (long k_ = 1; k_ <= n_; k_++) {                                              \
            g_count = 0;                                                                 \
            g_fail_at = k_;                                                              \
            int r_ = (call);                                                             \
            if (r_ != -2) fprintf(stderr, "allocation %ld of %ld: status %d\n", k_, n_, r_); \
            CHECK(r_ == -2);                                                             \
        }                                                                                \
        g_fail_at = 0;                                                                   \
    } while (0)

int main(void)
{
    orc_set_threads(2);
    const orc_scene s = make_scene();
    const int n = s.ntri;
    uint32_t ref_off[257];
    const int64_t nleaf = orc_leaf_refs(&s, ref_off);
    CHECK(nleaf > n);
    orc_bvh b;
    CHECK(alloc_bvh(&b, (int)nleaf));
    CHECK(orc_build_bvh(&s, &b) == 0);
    {
        float *boxes = malloc(sizeof(float) * 6 * (size_t)nleaf);
        uint32_t *rt = malloc(sizeof(uint32_t) * (size_t)nleaf);
        uint64_t *kc = malloc(sizeof(uint64_t) * (size_t)nleaf);
        CHECK(boxes && rt && kc);
        CHECK(orc_ref_boxes(&s, ref_off, boxes, rt) == 0);
        CHECK(orc_morton_boxes(boxes, nleaf, kc) == 0);
        EACH_ALLOCATION_FAILS(orc_morton_boxes(boxes, nleaf, kc));
        CHECK(orc_ref_boxes(&s, NULL, boxes, rt) == -1);
        CHECK(orc_morton_boxes(NULL, nleaf, kc) == -1);
        free(boxes);
        free(rt);
        free(kc);
    }
    CHECK(orc_leaf_refs(NULL, ref_off) == -1);

    /* closest hits: brute force and BVH agree */
    enum { NR = 512 };
    float org[3 * NR], dir[3 * NR], t0[NR], t1[NR];
    int32_t h0[NR], h1[NR];
    for (int i = 0; i < NR; i++) {
        org[3 * i] = 0.0f; org[3 * i + 1] = 1.2f; org[3 * i + 2] = 0.0f;
        dir[3 * i] = -0.5f + (float)(i % 32) / 32.0f;
        dir[3 * i + 1] = -0.4f + (float)(i / 32) / 32.0f;
        dir[3 * i + 2] = 1.0f;
    }
    CHECK(orc_closest_hit(&s, NULL, NR, org, dir, h0, t0) == 0);
    CHECK(orc_closest_hit(&s, &b, NR, org, dir, h1, t1) == 0);
    CHECK(memcmp(h0, h1, sizeof(h0)) == 0 && memcmp(t0, t1, sizeof(t0)) == 0);

    const orc_lens circle = {0.05f, 1.4f, 10.0f, 0.036f, 0, 0.0f};
    const orc_lens hexagon = {0.05f, 2.0f, 6.0f, 0.036f, 6, 0.2f};
    float zn = 0, zf = 0;
    CHECK(orc_zone(&circle, 64, &zn, &zf) == 0);
    CHECK(orc_coc(&circle, 64, 10.0f) == 0.0f);
    float lx = 0, ly = 0;
    CHECK(orc_lens_sample(1, 2, 3, 4, 6, 0.1f, &lx, &ly) == 0);
    float ox[81], oy[81], fr[81];
    orc_params pp = params(4, 0, 0, 1);
    CHECK(orc_gather_rings(&hexagon, &pp, ox, oy, fr) == 0);
    uint64_t codes[256];
    CHECK(orc_morton(&s, codes) == 0);

    const int W = 64, H = 48, m = 8;
    frame_bufs f;
    bufs_alloc(&f, W, H, m);
    const orc_camera c0 = camera(W, H, 0.0f, 0), c1 = camera(W, H, 0.03f, 1);
    CHECK(orc_gbuffer(&s, &b, &c0, &circle, f.colour, f.depth, f.normal) == 0);
    for (int mode = 0; mode < 4; mode++) {
        orc_params p = params(m, mode, 0, 0);
        CHECK(render(&s, &b, &f, &c0, &c1, &circle, &p, 1) == 0);
    }
    {
        orc_params p = params(m, 0, ORC_TAA_FINAL | ORC_TAA_RASTER | ORC_TAA_POST, 1);
        CHECK(render(&s, &b, &f, &c0, &c1, &hexagon, &p, 1) == 0);
    }
    uint32_t q[6] = {0, 17, 200, 511, 700, 767};
    float rgb[18];
    CHECK(orc_pixel_estimate(&s, &b, &c0, &circle, 6, q, 16, rgb) == 0);
    CHECK(orc_lens_integral(&s, &b, &c0, &hexagon, 6, q, 8, rgb) == 0);

    /* error paths: every allocation of the allocating entry points fails once */
    {
        orc_params p = params(m, 3, ORC_TAA_FINAL | ORC_TAA_RASTER | ORC_TAA_POST, 0);
        EACH_ALLOCATION_FAILS(orc_render_frame(&s, &b, &c0, &circle, NULL, NULL, 1, &p, f.colour, f.depth, f.normal,
                                               NULL, f.hist0, f.out, f.mask, NULL));
        orc_params p2 = params(m, 0, 0, 0);
        EACH_ALLOCATION_FAILS(orc_render_frame(&s, &b, &c1, &circle, &c0, &circle, 0, &p2, f.colour, f.depth,
                                               f.normal, f.hist0, f.hist1, f.out, f.mask, &f.dbg));
        EACH_ALLOCATION_FAILS(orc_build_bvh(&s, &b));
        EACH_ALLOCATION_FAILS(orc_morton(&s, codes));
    }
    /* invalid arguments */
    {
        orc_params p = params(0, 0, 0, 0);
        CHECK(orc_render_frame(&s, &b, &c0, &circle, NULL, NULL, 1, &p, f.colour, f.depth, f.normal, NULL, f.hist0,
                               f.out, f.mask, NULL) == -1);
        CHECK(orc_build_bvh(NULL, &b) == -1);
    }
    bufs_free(&f);
    free_bvh(&b);
    if (g_errors) {
        fprintf(stderr, "%d checks failed\n", g_errors);
        return 1;
    }
    printf("sanitize check ok: %d triangles\n", n);
    return 0;
}
