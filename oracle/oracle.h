/*
 * CPU oracle for the hybrid depth-of-field pass of Tan, Chua, Biette & Bhojan,
 * "A Hybrid System for Real-Time Rendering of Depth of Field Effect in Games".
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential restatement of
 * what the pass computes, used to check the GPU library.  Nothing in the
 * product path may link, load or call it; only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark do.
 *
 * It shares no code with the GPU library: its own structs, helpers, tables
 * and BVH.  It computes in IEEE binary32 with contraction disabled because
 * almost every stage ends in a discrete decision (a nearest texel, a ray
 * count, a closest triangle) that must be taken in the same precision as the
 * GPU kernels.  Functions whose arithmetic is not fixed by any independent
 * check say "parity unpinned" in their comment.
 *
 * Errors: every entry point returns 0 on success and a negative value on
 * invalid arguments; it never aborts.
 */
#ifndef DOF_ORACLE_H
#define DOF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    float pos[3], right[3], up[3], fwd[3]; /* orthonormal camera basis */
    int32_t width, height;                  /* full-resolution image size */
    uint32_t frame, seed;                   /* lens-sample counters */
    float jitter[2];                        /* sub-pixel sample offset, full-res pixels right/down (3.1.2) */
} orc_camera;

/* TAA stages (3.4): of the final image, of the raster image before
 * filtering, of the post-filter output. */
#define ORC_TAA_FINAL 1
#define ORC_TAA_RASTER 2
#define ORC_TAA_POST 4

typedef struct {
    float focal, fnum, focus, sensor;       /* f, N, d, w_s (scene units) */
    int32_t blades;                         /* 0 = circle, >= 3 polygon */
    float blade_rot;                        /* radians */
} orc_lens;

typedef struct {
    int32_t m;
    float s, var_mask_w, alpha, alpha_motion, var_recon_w, b_max, h_edge;
    float lod_scale, lod_max, depth_range, r_max;
    int32_t tile;
    float l_spec;
    int32_t mask_mode;                      /* 0 adaptive, 1 fixed, 2 all, 3 adaptive dilated by the neighbourhood max CoC */
    int32_t pp_polygon;                     /* 1: post-process gather taps on the aperture polygon (bladed lenses) */
    int32_t taa;                            /* TAA stages (3.4), bits ORC_TAA_*; history planes after the record */
    int32_t composite_literal;              /* 1: far-field blend read literally (high hit ratio -> post-process) */
} orc_params;

typedef struct {
    int32_t ntri;
    const float *verts;                     /* 9 per triangle */
    const float *albedo;                    /* 3 per triangle */
    float light_dir[3], light_rad[3], ambient[3], sky[3];
    int32_t leaf_split;                     /* s = 1..3: a long thin triangle becomes 2^s clipped leaf references; 0: none */
} orc_scene;

/* Binary radix tree over the leaf references (a triangle, or with
 * leaf_split one of its clipped pieces): 96-bit keys (the 64-bit key of the
 * reference's box -- a large-box flag over a 63-bit Morton code -- then the
 * reference index), Karras numbering.  All arrays are caller-allocated;
 * nleaf comes from orc_leaf_refs. */
typedef struct {
    int32_t nleaf;
    uint64_t *keys;         /* nleaf 64-bit keys, ascending with refs */
    uint32_t *refs;         /* nleaf reference indices in leaf order */
    uint32_t *ids;          /* nleaf triangle ids in leaf order */
    uint32_t *left, *right; /* nleaf-1 each; bit 31 set = leaf (sorted index) */
    uint32_t *parent;       /* 2*nleaf-1: internal nodes then leaves; root = ~0u */
    float *bounds;          /* 6 per internal node: lo xyz, hi xyz */
    float *leaf_bounds;     /* 6 per leaf, sorted order */
} orc_bvh;

typedef struct {
    float *colr;        /* A1: hw*hh*4 (half-res colour rgb, signed radius) */
    float *zn;          /* A1: hw*hh*4 (min depth, its normal xyz) */
    float *tile_max;    /* A2: tw*th */
    float *tile_dil;    /* A2: tw*th */
    float *pre;         /* A3: hw*hh*4 */
    float *gather;      /* A4: hw*hh*4 (v_p rgb, bokeh proportion) */
    float *ppmed;       /* A5: hw*hh*4 */
    int32_t *prev_idx;  /* A6: hw*hh reprojected texel or -1 */
    uint32_t *queue;    /* A7: hw*hh */
    uint32_t *ray_base; /* A7: hw*hh */
    int32_t *ray_hit;   /* A10: hw*hh*m */
    float *ray_t;       /* A10: hw*hh*m */
    float *ray_col;     /* A10: 4 per ray (rgb, view depth) */
    float *ray_pos;     /* A10: 4 per ray (xyz, 0) */
    float *resolve;     /* A11: 4 planes of hw*hh*4 */
    float *temporal;    /* A12: 2 planes of hw*hh*4 */
    float *var_blur;    /* A12: hw*hh */
    float *rtmed;       /* A13: hw*hh*4 */
    float *mips;        /* A13: levels 0..3 back to back, 4 per texel */
    float *recon;       /* A13: hw*hh*4 (c_rec rgb, h_rec) */
    int64_t n_masked, n_rays;
} orc_debug;

void orc_set_threads(int n);
int orc_threads(void);

float orc_coc(const orc_lens *lens, int32_t width, float z);
int orc_zone(const orc_lens *lens, int32_t width, float *z_near, float *z_far);

int orc_morton(const orc_scene *s, uint64_t *codes);

/* Leaf references (early split clipping, Ernst & Greiner 2007): ref_off gets
 * ntri+1 offsets (triangle i owns references ref_off[i] .. ref_off[i+1]-1);
 * returns their number, or < 0 on bad arguments. */
int64_t orc_leaf_refs(const orc_scene *s, uint32_t *ref_off);

/* The references' boxes (6 floats: lo xyz, hi xyz) and triangles. */
int orc_ref_boxes(const orc_scene *s, const uint32_t *ref_off, float *boxes, uint32_t *ref_tri);

/* orc_morton's keys for n boxes given as lo xyz, hi xyz. */
int orc_morton_boxes(const float *boxes, int64_t n, uint64_t *codes);
int orc_build_bvh(const orc_scene *s, orc_bvh *b);

/* Closest hit per ray; bvh == NULL means brute force over all triangles. */
int orc_closest_hit(const orc_scene *s, const orc_bvh *b, int64_t nrays,
                    const float *org, const float *dir, int32_t *hit, float *t);

int orc_lens_sample(uint32_t seed, uint32_t frame, uint32_t q, uint32_t k,
                    int32_t blades, float blade_rot, float *lx, float *ly);

int orc_gbuffer(const orc_scene *s, const orc_bvh *b, const orc_camera *cam,
                const orc_lens *lens, float *colour, float *depth, float *normal);

/* The post-process gather's 81 taps (offsets in kernel radii, ring
 * distances): circles, or the aperture polygon with params->pp_polygon. */
int orc_gather_rings(const orc_lens *lens, const orc_params *p, float *ox, float *oy, float *frac);

int orc_render_frame(const orc_scene *s, const orc_bvh *b,
                     const orc_camera *cam, const orc_lens *lens,
                     const orc_camera *prev_cam, const orc_lens *prev_lens,
                     int32_t reset, const orc_params *p,
                     const float *gb_colour, const float *gb_depth,
                     const float *gb_normal, const float *hist_in,
                     float *hist_out, float *out_colour, uint8_t *out_mask,
                     orc_debug *dbg);

/* Mean colour of spp thin-lens rays through half-res pixels (estimator). */
int orc_pixel_estimate(const orc_scene *s, const orc_bvh *b,
                       const orc_camera *cam, const orc_lens *lens,
                       int64_t nq, const uint32_t *qlist, int32_t spp,
                       float *rgb);

/* Stratified G x G lens-grid quadrature of the same pixels (reference). */
int orc_lens_integral(const orc_scene *s, const orc_bvh *b,
                      const orc_camera *cam, const orc_lens *lens,
                      int64_t nq, const uint32_t *qlist, int32_t grid,
                      float *rgb);

#ifdef __cplusplus
}
#endif
#endif
