/*
 * libdof -- hybrid depth-of-field pass for AMD Instinct MI355X (gfx950).
 *
 * Implements the per-frame pass of Tan, Chua, Biette & Bhojan, "A Hybrid
 * System for Real-Time Rendering of Depth of Field Effect in Games":
 * a post-process gather blur (section 3.1), thin-lens rays traced only where
 * a ray mask asks for them (3.2.1-3.2.2), temporal and spatial reconstruction
 * of those sparse samples (3.2.3-3.2.4) and the adaptive composite of both
 * (3.3).  Every stage is a HIP kernel; this header is the whole interface.
 *
 * Conventions
 *  - Plain C.  Every call returns a dof_status; 0 is success.  On failure
 *    dof_last_error() returns a message for the calling thread.  No C++
 *    exception crosses this boundary.
 *  - "device pointer" means memory on the current HIP device; "host pointer"
 *    means ordinary host memory.  The library never allocates device memory:
 *    the caller owns every device buffer (scene arena, history, outputs,
 *    scratch) and sizes it with the *_bytes() queries.  Host structs are
 *    read during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All device work is enqueued on it; no call synchronises the device
 *    except where stated.  Asynchronous device faults surface as
 *    DOF_E_DEVICE on a later call.
 *  - Images are row-major, row 0 at the top; pixel (x, y) is at y * W + x.
 *    Full-resolution W and H must be even; half resolution is W/2 x H/2.
 *  - Camera: orthonormal right/up/forward, view depth z = (P - pos) . fwd;
 *    pixel (x, y) looks along fwd + u right + v up with
 *    u = (2 (x + 1/2) / W - 1) tan_x, v = (1 - 2 (y + 1/2) / H) tan_y,
 *    tan_x = w_s (d - f) / (2 f d) (sensor at the focused image distance),
 *    tan_y = tan_x H / W.
 *  - A dof_scene must not be used from two threads at once; distinct scenes
 *    may be.
 */
#ifndef DOF_H
#define DOF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DOF_ABI_VERSION 6

typedef int32_t dof_status;
#define DOF_OK 0
#define DOF_E_INVALID 1     /* bad argument: null pointer, size, format, range */
#define DOF_E_NOMEM 2       /* a caller-provided buffer is too small */
#define DOF_E_DEVICE 3      /* a HIP call failed (message in dof_last_error) */
#define DOF_E_STATE 4       /* call out of order, e.g. render before build */
#define DOF_E_UNSUPPORTED 5 /* valid but not implemented (e.g. tile != 16) */

#define DOF_RGBA32F 0       /* 4 x float per pixel, 16 B */
#define DOF_RGBA16F 1       /* 4 x IEEE half per pixel, 8 B */

#define DOF_MASK_ADAPTIVE 0 /* ray count from eqs. (2)-(4) */
#define DOF_MASK_FIXED 1    /* m rays wherever the adaptive count is > 0 */
#define DOF_MASK_ALL 2      /* m rays at every half-res pixel */
/* the adaptive counts grown by the neighbourhood's maximum CoC (the remedy
 * section 5.3 proposes for tiling near the camera): each pixel takes the
 * largest count within a square window whose radius is its tile's dilated
 * maximum CoC radius, rounded up (r_max must be <= 32 in this mode) */
#define DOF_MASK_DILATE 3

/* Bits of dof_params.taa: temporal anti-aliasing stages (section 3.4, after
 * Karis 2014).  Each blends an image with its previous version at the
 * reprojected position, that history clamped per RGB channel to the current
 * 3 x 3 range, history weight 0.9; each keeps its previous version in its
 * own plane of the history buffer. */
#define DOF_TAA_FINAL 1     /* the output, after the composite */
#define DOF_TAA_RASTER 2    /* the G-buffer colour, before any filtering; every later stage reads the result */
#define DOF_TAA_POST 4      /* the half-res post-filter output, before the composite reads it */

typedef struct {
    float pos[3], right[3], up[3], fwd[3];
    int32_t width, height;  /* full resolution */
    uint32_t frame, seed;   /* counters of the lens-sample hash */
    /* sub-pixel camera jitter (section 3.1.2): this frame's sample positions
     * sit (jitter[0], jitter[1]) full-res pixels right of and below the pixel
     * centres, for the G-buffer rays, the traced rays and the reconstruction
     * of world points from depth; |jitter| <= 1.  Projections into the
     * previous view ignore its jitter (histories are unjittered images). */
    float jitter[2];
} dof_camera;

/* Thin lens (sections 1.1, 3.3): focal length f, f-number N (aperture
 * diameter a = f / N; N = +inf gives a pinhole), focus distance d, sensor
 * width w_s, all in scene units.  blades = 0 for a circular aperture, else a
 * regular polygon with 3..16 blades rotated by blade_rot radians. */
typedef struct {
    float focal, fnum, focus, sensor;
    int32_t blades;
    float blade_rot;
} dof_lens;

/* Every tunable of the pass, with the paper's values as defaults
 * (dof_default_params).  m: ray budget per pixel (3.2.1), 1..255.
 * s: eq. (2) scale (4.2).  var_mask_w: eq. (4) weight (1e5).  alpha: history
 * weight of the moving average (0.95, 3.2.3); alpha_motion: reduced weight
 * when the camera moved.  var_recon_w, b_max: eq. (5).  h_edge: eq. (7).
 * lod_scale, lod_max: eq. (8).  depth_range: main-filter depth range (0.1 =
 * 10 cm, 4.2).  r_max: largest gather radius in half-res pixels.  tile:
 * neighbourhood-max tile side (16 only).  l_spec: luma above which a gather
 * tap counts as a bright, specular sample (3.1.2).  trace_blocks: blocks of
 * 128 threads of the persistent traversal kernel, at most 4096 (0 = as many
 * as are resident at once).  timing: see dof_stage_times. */
typedef struct {
    uint32_t struct_size;   /* = sizeof(dof_params) */
    int32_t m;
    float s, var_mask_w, alpha, alpha_motion, var_recon_w, b_max, h_edge;
    float lod_scale, lod_max, depth_range, r_max;
    int32_t tile;
    float l_spec;
    int32_t mask_mode;
    int32_t trace_blocks;
    int32_t timing;         /* nonzero: record a HIP event pair per stage */
    /* 1: with a bladed lens, the post-process gather samples the aperture
     * polygon instead of circles (section 2 names polygonal bokeh as a
     * change of the sampling kernel's shape); 0 (default): circles */
    int32_t pp_polygon;
    /* TAA stages, bits DOF_TAA_* (0 = none).  A stage's previous image lives
     * in the history buffer; turning a stage on mid-sequence needs
     * history.reset. */
    int32_t taa;
    /* 1: keep each traced ray's hit id, distance, shaded colour and hit
     * position in the scratch (40 more bytes per ray of half-res pixels x m)
     * for dof_debug_view_get; 0 (default): the shading writes none of them */
    int32_t ray_records;
    /* Section 3.3 says both that a high hit ratio favours the post-process
     * colour and that the blend happens only below a hit ratio of 0.3 because
     * leaning to post-processing above it loses the ray-traced
     * semi-transparencies.  0 (default): far-field output = lerp(post-process,
     * ray traced, smoothstep(0, h_edge, h)); 1: the first sentence read
     * literally, lerp(ray traced, post-process, smoothstep(0, h_edge, h)). */
    int32_t composite_literal;
    /* Launch-shape knobs, searched by the autotuner (0 = library default);
     * no result depends on them.  gather_window: side of the LDS window in
     * which the post-process gather stages the texels of each tile whose taps
     * fit it, 32, 40 or 48, or -1 (and the default 0): every tap read from
     * global memory.  trace_stack:
     * LDS traversal stack entries per lane, 16, 24 (default) or 32.
     * trace_grab: rays a wave takes from the traversal's work counters at a
     * time, 1..256 (default 64).  trace_refill: idle lanes at which a wave takes
     * new rays, 1..64 (default 16).  trace_leaf_batch: lanes with a pending
     * leaf at which a wave runs its triangle tests, 1..64 (default 32).
     * trace_order: the order in which the persistent traversal hands out the
     * rays of the queue (row-major pixels): 1 from the first ray, 2 (and the
     * default 0) from the last -- the bottom image rows first, which in
     * ground-level views holds the near foreground whose rays cost most, so
     * cheap sky and background rays fill the kernel's tail.  trace_steps:
     * node visits per lane in one iteration of the traversal loop (between
     * its refill and triangle-test decisions), 3 or 4 (and the default 0). */
    int32_t gather_window;
    int32_t trace_stack;
    int32_t trace_grab;
    int32_t trace_refill;
    int32_t trace_leaf_batch;
    int32_t trace_order;
    int32_t trace_steps;
} dof_params;

/* Full-resolution G-buffer (section 3): sharp colour (alpha ignored), view
 * depth (+inf for the sky), world normal xyz (w ignored).  Device pointers. */
typedef struct {
    const void *colour;
    int32_t colour_format;  /* DOF_RGBA32F or DOF_RGBA16F */
    const float *depth;
    const void *normal;
    int32_t normal_format;
} dof_gbuffer;

/* Temporal history (3.2.3): dof_history_bytes() per buffer.  `in` is last
 * frame's `out` (ignored when reset != 0); `out` is written completely
 * (a TAA plane only when its stage is on).  in and out must not overlap.
 * prev_camera / prev_lens: the view of `in`.  Layout: the half-res record,
 * four planes back to back -- float4 (near rgb, hit ratio), float4 (far rgb,
 * age), float4 (near CoC, far CoC, luma mean, luma second moment), float
 * (blurred luma variance) -- then, from the record's size rounded up to 16
 * bytes, the TAA planes of float4 per pixel: the final output (full res),
 * the raster colour (full res), the post-filter output (half res). */
typedef struct {
    const void *in;
    void *out;
    dof_camera prev_camera;
    dof_lens prev_lens;
    int32_t reset;
} dof_history_io;

/* Device-side counters of one frame. */
typedef struct {
    uint32_t masked_px;     /* half-res pixels with at least one ray */
    uint32_t rays;          /* thin-lens rays traced */
    uint64_t node_visits;   /* BVH nodes fetched by the traversal */
    uint64_t tri_tests;     /* ray/triangle tests */
    uint32_t stack_spills;  /* times a lane's LDS traversal stack was full and dropped its 8 oldest
                             * entries (found again through parent links; the result is unchanged) */
    uint32_t reserved[1];
} dof_stats;

typedef struct {
    void *colour;           /* device, W x H, colour_format */
    int32_t colour_format;
    uint8_t *mask;          /* device, W/2 x H/2 ray counts (the ray mask) */
    dof_stats *stats;       /* device, may be NULL */
} dof_frame_out;

typedef struct {
    int32_t ntri;
    const float *verts;     /* host, 9 floats per triangle (v0 v1 v2 xyz) */
    const float *albedo;    /* host, 3 floats per triangle */
    float light_dir[3];     /* direction the light travels (unit) */
    float light_rad[3], ambient[3], sky[3];
    int32_t leaf_split;     /* s = 1..3: a long thin triangle (its box's three face areas sum to more
                             * than 8 times its area) becomes 2^s leaf references, the triangle clipped
                             * to equal slabs of its box along the longest axis (early split clipping,
                             * Ernst & Greiner 2007), so rays that enter the box beside the triangle
                             * mostly skip its test; 0: one leaf per triangle.  Hits are the same;
                             * which s is fastest depends on the scene. */
} dof_scene_desc;

typedef struct dof_scene dof_scene;

/* Device views of the acceleration structure (for inspection and tests).
 * Its nleaf leaves are references: a triangle, or with leaf_split one of the
 * 2^leaf_split pieces of a split triangle; reference r of triangle i is
 * ref_off[i] + j (pieces j in slab order), and its box is the
 * triangle's box, or for a piece: on the split axis the slab, on the others
 * the range of the piece's vertices and edge crossings (each crossing
 * widened by 2^-20 (|edge extent| + |x|)), clipped to the triangle's box.
 * keys: sorted 64-bit keys, ties in reference order: bits 0-62 are the
 * Morton code of the reference box centre on cubic cells (one scale, 2^21
 * over the largest extent of the centre bounds; 21 bits per axis, x at bit
 * 3i+2, y 3i+1, z 3i), bit 63 is set for a box whose diagonal exceeds a
 * quarter of the centre bounds' diagonal; ids: reference indices in that
 * order; nodes: nleaf-1 records of 64 B {float4 (L.lo.x, L.hi.x, L.lo.y,
 * L.hi.y), float4 (R.lo.x, R.hi.x, R.lo.y, R.hi.y), float4 (L.lo.z, L.hi.z,
 * R.lo.z, R.hi.z), uint4 (left, right, first leaf, last leaf)}, child bit
 * 31 = leaf (sorted index), the node covering the sorted leaves
 * first..last; parent: 2 nleaf - 1 entries (internal nodes, then leaves),
 * root = ~0u; tris: 3 float4 per leaf in sorted order, the vertices of the
 * leaf's triangle (w of the first = triangle id bits); nodes16: the copy of
 * the nodes the traversal reads, nleaf-1 records of 32 B {uint32 L.x, L.y,
 * L.z, R.x, R.y, R.z, left, right}, each box axis a binary16 pair (low plane
 * in bits 0-15 rounded down, high plane in bits 16-31 rounded up; a result
 * in the subnormal range moved outward to 0 or to 2^-14), so each box holds
 * the binary32 one. */
typedef struct {
    int32_t ntri;
    int32_t nleaf;
    const uint64_t *keys;
    const uint32_t *ids, *parent;
    const void *nodes, *tris;
    const void *nodes16;
} dof_bvh_view;

/* Device pointers into a frame's scratch (valid after dof_render_frame);
 * ray_hit, ray_t, ray_col and ray_pos are NULL unless params.ray_records. */
typedef struct {
    void *colr, *zn, *tile_max, *tile_dil, *pre, *gather, *ppmed, *prev_idx;
    void *queue, *ray_base, *ray_hit, *ray_t, *ray_col, *ray_pos;
    void *resolve, *temporal, *var_blur, *rtmed, *mips, *recon, *counters;
} dof_debug_view;

int32_t dof_abi_version(void);
const char *dof_last_error(void);
void dof_default_params(dof_params *p);

/* Scene arena size bound for ntri triangles of any shape: input triangles,
 * then per leaf reference (at most 8 per triangle) its box, the leaf-ordered
 * triangle, BVH node and parent links, and the build's keys, sort buffers and
 * counters (about 200 bytes per reference). */
dof_status dof_scene_bytes(int32_t ntri, size_t *bytes);

/* The exact arena size for desc's triangles (counts the split triangles
 * when desc->leaf_split); errors as dof_create_scene's argument checks. */
dof_status dof_scene_bytes_desc(const dof_scene_desc *desc, size_t *bytes);

/* Copies desc's host arrays into `arena` (device, >= dof_scene_bytes_desc) on
 * `stream` and returns a host handle; the arena must outlive the scene.
 * Synchronises `stream` once (the host arrays may be freed on return). */
dof_status dof_create_scene(const dof_scene_desc *desc, void *arena, size_t arena_bytes,
                            void *stream, dof_scene **out);

/* LBVH build on the device (Morton codes, radix sort, binary radix tree,
 * bottom-up bounds) -- the acceleration structure the paper builds with DXR
 * inside its Ray Trace timing (5.2). */
dof_status dof_build_bvh(dof_scene *scene, void *stream);
dof_status dof_bvh_view_get(const dof_scene *scene, dof_bvh_view *out);
void dof_destroy_scene(dof_scene *scene);

/* Closest hit of n rays (device arrays org[3n], dir[3n]; dir need not be
 * unit) -> hit[n] original triangle id or -1, t[n] distance or +inf. */
dof_status dof_trace_rays(const dof_scene *scene, int64_t n, const float *org, const float *dir,
                          int32_t *hit, float *t, void *stream);

/* All-in-focus G-buffer through the lens centre, one ray per full-res pixel
 * (the sharp raster image of section 3, produced here by ray casting). */
dof_status dof_render_gbuffer(const dof_scene *scene, const dof_camera *cam, const dof_lens *lens,
                              void *colour, int32_t colour_format, float *depth, void *normal,
                              int32_t normal_format, void *stream);

/* Ground truth of the accuracy judge (section 5.1 measures the hybrid
 * against full ray tracing): the thin-lens estimate of every full-res pixel,
 * the mean shaded colour of spp rays from lens points towards the pixel's
 * point on the focus plane (section 3.2.2's ray model at full resolution).
 * Ray k of pixel y * W + x uses the lens sample the pass would give
 * half-res pixel q = y * W + x of a 2W x 2H frame, so an oracle estimate over
 * the same counters reproduces it.  Sums each pixel's colours in binary64 in
 * sample order.  colour: device, W x H in colour_format (alpha 1).
 * scratch: device, >= dof_reference_scratch_bytes (the (leaf, t) records of
 * one chunk of at most 2^22 rays, whole pixels).  spp: 1..1024.  Uses the
 * scene's work counter, like dof_render_gbuffer: not concurrently with
 * another call on the same scene. */
dof_status dof_reference_scratch_bytes(int32_t width, int32_t height, int32_t spp, size_t *bytes);
dof_status dof_render_reference(dof_scene *scene, const dof_camera *cam, const dof_lens *lens, int32_t spp,
                                void *colour, int32_t colour_format, void *scratch, size_t scratch_bytes,
                                void *stream);

dof_status dof_history_bytes(int32_t width, int32_t height, size_t *bytes);
dof_status dof_history_reset(void *hist, int32_t width, int32_t height, void *stream);
/* Scratch of one frame.  A frame may ask for at most 2^31 rays (half-res
 * pixels x params.m): ray indices and counters are 32-bit; beyond it this
 * query, dof_render_frame and dof_batch_set return DOF_E_UNSUPPORTED. */
dof_status dof_frame_scratch_bytes(int32_t width, int32_t height, const dof_params *p, size_t *bytes);

/* The pass (sections 3.1-3.4) for one frame: CoC and half-res reduce, tile
 * max, prefilter, 81-tap gather, median, ray mask, compaction and thin-lens
 * ray generation, traversal, shading of the hits and resolve, temporal
 * accumulation, variance blur, median + mips, reconstruction, composite, and
 * the TAA stages params.taa selects.  Enqueued on `stream`, no host sync.
 * Unless params.timing is set, the post-process chain (tile dilation but in
 * the dilated mask mode, prefilter, gather, median) runs on a stream the
 * scene owns (created with it, default priority), forked from `stream` after
 * the ray generation (it reads only what the reduce wrote) and joined back
 * before the composite with events, so it runs beside the traversal: the
 * work stays ordered on `stream` and a HIP graph capture of the call takes
 * both branches.  Frames of one scene share that stream, so their
 * post-process chains run one after another. */
dof_status dof_render_frame(dof_scene *scene, const dof_camera *cam, const dof_lens *lens,
                            const dof_gbuffer *gb, const dof_history_io *hist, const dof_params *p,
                            const dof_frame_out *out, void *scratch, size_t scratch_bytes,
                            void *stream);

/* dof_render_frame without a caller scratch buffer, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The scratch is a buffer of
 * DOF_NOALLOC_SCRATCH_MB MiB that the library keeps on each GPU it runs on
 * until the process ends; this call allocates nothing.  Frames whose
 * dof_frame_scratch_bytes exceeds it (e.g. 640 x 360 at m = 8 fits, 1920 x
 * 1080 does not) and params.timing != 0 return DOF_E_UNSUPPORTED; everything
 * else behaves as dof_render_frame.  Every call on a GPU shares that GPU's
 * buffer: calls that overlap on one GPU (two streams or two threads) race,
 * and the per-frame planes of dof_debug_view_get are only those of the last
 * call.  The buffer's device address is looked up on the first call on each
 * device (outside a stream capture, preferably). */
#define DOF_NOALLOC_SCRATCH_MB 64
dof_status dof_render_frame_noalloc(dof_scene *scene, const dof_camera *cam, const dof_lens *lens,
                                    const dof_gbuffer *gb, const dof_history_io *hist, const dof_params *p,
                                    const dof_frame_out *out, void *stream);

/* Stages timed when params.timing is set, in launch order. */
#define DOF_NUM_STAGES 13
/* Per-stage device time (ms) of the scene's most recent frame rendered with
 * params.timing != 0: reduce (with the raster TAA), dilate, prefilter,
 * gather, median (with the post-filter TAA), mask, compaction (with the ray
 * generation), trace (the traversal alone), resolve (with the shading),
 * temporal, blur+median+mips, reconstruction, composite (with the final TAA).  Waits for that frame's last event (host sync on it only).
 * Writes min(cap, DOF_NUM_STAGES) values to ms (host) and the count to *n. */
dof_status dof_stage_times(dof_scene *scene, float *ms, int32_t cap, int32_t *n);

dof_status dof_debug_view_get(void *scratch, int32_t width, int32_t height, const dof_params *p,
                              dof_debug_view *out);

/* ---- Batches: frames of several sessions in one launch per stage --------
 * Not a passage of the paper (it renders one view per frame): a throughput
 * path for serving many sessions at once.  Each item is one frame with the
 * same arguments as dof_render_frame (its own scene, size, G-buffer,
 * history, outputs and scratch); all items share one dof_params.  Every
 * stage runs as one launch over all items' pixels and one persistent
 * traversal runs over all items' rays, and each item's colour, mask,
 * history and scratch planes are bit-identical to what dof_render_frame
 * gives for it alone.  Items of one batch must not share a scratch,
 * history output or colour buffer.  params.timing is ignored. */
#define DOF_MAX_BATCH 128

typedef struct dof_batch dof_batch;

typedef struct {
    dof_scene *scene;
    dof_camera camera;
    dof_lens lens;
    dof_gbuffer gbuffer;
    dof_history_io history;
    dof_frame_out out;          /* out.stats: masked_px and rays of this item, visits/tests 0 */
    void *scratch;              /* dof_frame_scratch_bytes(width, height, params) bytes */
    size_t scratch_bytes;
} dof_batch_item;

/* Device-written totals of one batch run. */
typedef struct {
    int32_t frames;
    uint32_t rays;
    uint64_t node_visits;
    uint64_t tri_tests;
} dof_batch_stats;

/* Size of the device table of a batch of up to max_items (<= DOF_MAX_BATCH). */
dof_status dof_batch_bytes(int32_t max_items, size_t *bytes);
/* Host handle over a caller-owned device table (256-byte aligned, at least
 * dof_batch_bytes(max_items) bytes, kept alive until dof_batch_destroy). */
dof_status dof_batch_create(void *table, size_t table_bytes, int32_t max_items, dof_batch **out);
/* Checks every item as dof_render_frame would (an error names the item) and
 * uploads the item table on `stream` (host memory is not retained). */
dof_status dof_batch_set(dof_batch *b, const dof_batch_item *items, int32_t n, const dof_params *p,
                         void *stream);
/* Renders the items of the last dof_batch_set on `stream`: launches only
 * (no host sync, no allocation), so it may be captured in a HIP graph.  A
 * captured run may be replayed after later dof_batch_set calls whose items
 * have the same count, sizes and order (grid sizes are captured).  As in
 * dof_render_frame, the post-process chain runs on a stream the batch owns
 * (created with it, default priority), forked from `stream` after the ray
 * generation and joined back before the composite; runs of one batch share
 * it.  stats (device pointer, nullable) receives the batch totals. */
dof_status dof_batch_run(dof_batch *b, dof_batch_stats *stats, void *stream);
void dof_batch_destroy(dof_batch *b);

#ifdef __cplusplus
}
#endif
#endif
