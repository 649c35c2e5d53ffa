// Internal declarations shared by the libdof translation units (not part of
// the ABI).  Device helpers here are compiled with contraction off and
// correctly rounded division/sqrt, so every kernel computes in plain
// IEEE binary32 in the order written.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/dof.h"

namespace dof {

constexpr uint32_t kLeaf = 0x80000000u;
constexpr float kSqrt2 = 1.41421356237f;  // one pixel diagonal (3.1.1, 3.3)
constexpr int kTile = 16;                 // neighbourhood-max tile side
constexpr int kRingTaps = 81;             // 1 + 8 + 16 + 24 + 32 (3.1.1)
constexpr int kMaxBlades = 16;
constexpr int kStackLds = 24;             // default traversal stack entries per lane (LDS only; deeper
                                          // work is found again through parent links); 16 and 32 also built
constexpr int kTB = 128;                  // threads per traversal block
constexpr int kTraceSteps = 4;            // default node visits per lane in one traversal loop iteration
constexpr int kMaxTraceBlocks = 4096;     // persistent traversal grid limit

// ---------------------------------------------------------------- scene

struct BvhNode {      // 64 B, both children's boxes with the parent
    float4 a;         // L.lo.x, L.hi.x, L.lo.y, L.hi.y
    float4 b;         // R.lo.x, R.hi.x, R.lo.y, R.hi.y
    float4 c;         // L.lo.z, L.hi.z, R.lo.z, R.hi.z
    uint4 d;          // left, right, first and last leaf of the range (bit 31 of a child: leaf)
};

// The traversal's copy of a node, 32 B: the children's boxes in binary16,
// each low plane rounded down and each high plane rounded up (no subnormal
// values: those go out to 0 or to the smallest normal), so every box holds the
// binary32 box and the slab test stays conservative.  Each 32-bit word packs
// one axis of one box: the low plane in its low half, the high plane in its
// high half.
struct BvhNode16 {
    uint4 a;          // L.x, L.y, L.z, R.x
    uint4 b;          // R.y, R.z, left, right
};

struct SceneShade {
    float light_dir[3], light_rad[3], ambient[3], sky[3];
};

// The tree's leaves are references: a triangle, or (early split clipping)
// one of four pieces of a long thin triangle clipped to quarters of its box.
struct SceneDev {
    int32_t ntri;
    int32_t nleaf;           // references
    const float *verts_in;   // 9 per triangle, original order
    const float *albedo_in;  // 3 per triangle, original order
    const uint32_t *ref_off; // ntri + 1: triangle i owns references ref_off[i] .. ref_off[i+1]-1
    float *ref_box;          // 6 per reference: lo xyz, hi xyz
    uint32_t *ref_tri;       // triangle of each reference
    float4 *tris;            // 3 per leaf, sorted order; tris[3i].w = triangle id bits
    float4 *albedo;          // 1 per leaf, sorted order
    BvhNode *nodes;          // nleaf - 1
    BvhNode16 *nodes16;      // nleaf - 1: the traversal's binary16 copy
    uint32_t *parent;        // 2 nleaf - 1
    uint64_t *keys, *keys_tmp;   // 63-bit Morton codes
    uint32_t *ids, *ids_tmp;     // reference indices (sorted: in leaf order)
    uint32_t *flags;         // nleaf - 1 refit visit counters
    uint32_t *hist;          // radix histograms (digit-major) + 256 digit offsets
    float *bounds;           // 6 partial-bound slots per reduce block + 8 final
    uint32_t *aux;           // work counters of the scene-level traversal kernels ([8]: the refit's exit count)
    int32_t sort_blocks;
    int32_t bound_blocks;
};

// ---------------------------------------------------------------- frame

struct Aperture {
    int32_t blades;
    float apothem;
    float nx[kMaxBlades], ny[kMaxBlades];
};

struct Rings {
    float ox[kRingTaps], oy[kRingTaps], frac[kRingTaps];
};

struct ViewConst {    // a camera with its lens-derived projection
    float pos[3], right[3], up[3], fwd[3];
    float tanx, tany;
    float ju, jv;     // camera jitter as an offset of normalised image coordinates (0 for a previous view)
};

// View direction through the (jittered) centre of pixel (x, y) of a w x h grid.
__device__ inline void pixel_dir(const ViewConst &v, int x, int y, int w, int h, float fv[3])
{
    float u = (((((float)x + 0.5f) * 2.0f) / (float)w - 1.0f) + v.ju) * v.tanx;
    float vv = ((1.0f - (((float)y + 0.5f) * 2.0f) / (float)h) - v.jv) * v.tany;
#pragma unroll
    for (int a = 0; a < 3; ++a) fv[a] = (v.fwd[a] + u * v.right[a]) + vv * v.up[a];
}

// Launch-shape knobs of the traversal (dof_params.trace_*; results do not
// depend on them).
struct TraceKnobs {
    int32_t stack;        // LDS stack entries per lane: 16, 24 or 32
    uint32_t grab;        // rays per take from the work counters
    int32_t refill;       // idle lanes that trigger a refill
    int32_t leaf_batch;   // lanes with a pending leaf that trigger the triangle tests
    int32_t reverse;      // 1: rays handed out from the end of the queue
    int32_t steps;        // node visits per lane in one loop iteration: 3 or 4
};

struct FrameConst {
    int32_t W, H, hw, hh, tw, th, T, D;
    int32_t gather_win;       // LDS window side of the gather (0: none)
    TraceKnobs tk;
    int32_t m, mask_mode, have_hist, motion, taa, ray_records, composite_literal;
    uint32_t seed, frame;
    float d, half_a, cock, znb, ramp;
    float s, var_mask_w, alpha_h, var_recon_w, b_max, h_edge, lod_scale, lod_max, depth_range;
    float r_max, l_spec;
    int32_t lod_levels;       // highest mip level used (<= 3)
    ViewConst cur, prev;
    Aperture ap;
    SceneShade shade;
    int32_t mw[4], mh[4];     // mip level sizes
    int64_t moff[4];          // mip level offsets in float4 units
};

// Byte offsets of every plane in a frame's scratch buffer.
struct ScratchLayout {
    size_t colr, zn, zh, tile_max, tile_dil, pre, gather, ppmed, prev_idx, mask_raw;
    size_t chunk_cnt, chunk_off, counters;
    size_t queue, ray_base, ray_pix, ray_rec, ray_lt, ray_hit, ray_t, ray_col, ray_pos;
    size_t gtex, resolve, temporal, var_blur, rtmed, mips, tap, recon, comp, rast, pptaa;
    size_t total;
    int64_t nchunks;
};

constexpr int kChunk = 1024;   // pixels per compaction chunk (256 threads x 4)

// Device pointers of every plane of one frame (from its scratch layout).
struct Planes {
    float4 *colr, *zn, *pre, *gather, *ppmed;
    float *zh, *tile_max, *tile_dil;
    int32_t *prev_idx;
    uint2 *chunk_cnt, *chunk_off;
    uint32_t *counters, *queue, *ray_base, *ray_pix;
    int32_t *ray_hit;        // per-ray planes: nullptr unless params.ray_records
    float *ray_t;
    float4 *ray_col, *ray_pos;
    float4 *rec0;                 // ray records: (o, d.x) per ray
    float2 *rec1;                 //              (d.y, d.z) per ray
    uint2 *ray_lt;                // traversal result per ray: (leaf of the hit or ~0, t bits)
    float4 *R0, *R1, *R2, *R3, *T0, *T1, *rtmed, *mips, *recon;
    float *var_blur;
    float2 *tap;             // per half-res pixel: (CoC if ray traced else -inf, hit ratio)
    float4 *gtex;            // per half-res pixel, as the gather reads it: prefiltered rgb and |CoC radius|,
                             // the radius's sign bit set for a bright (specular) pixel
    uint8_t *mask_raw;       // adaptive ray counts before dilation (mask mode DOF_MASK_DILATE)
    float4 *comp;            // full-res composite colour before the final TAA (DOF_TAA_FINAL)
    float4 *rast;            // full-res raster colour after its TAA (DOF_TAA_RASTER)
    float4 *pptaa;           // half-res post-filter output after its TAA (DOF_TAA_POST)
    float4 *ppout;           // what the composite reads: pptaa with DOF_TAA_POST, else ppmed
};
Planes planes(const FrameConst &fc, const ScratchLayout &L, char *scratch);
// The G-buffer as the stages after the raster TAA read it: with
// DOF_TAA_RASTER its colour is the resolved plane (RGBA32F), else gb itself.
dof_gbuffer resolved_gbuffer(const FrameConst &fc, const Planes &P, const dof_gbuffer &gb);

// What the traversal reads of a scene.
struct SceneArgs {
    int32_t nleaf;
    const float4 *__restrict__ tris;
    const float4 *__restrict__ albedo;
    const BvhNode16 *__restrict__ nodes;   // binary16 boxes (conservative)
    const uint32_t *__restrict__ parent;   // parent of each internal node (root: ~0u)
};

// ---------------------------------------------------------------- batches
// A batch renders several frames (any scenes and sizes) with one launch per
// stage: every stage kernel runs over the concatenation of the frames'
// block grids, and one persistent traversal runs over the concatenation of
// their ray queues.  The device table holds a BatchHead and one Job per frame.

constexpr int kMaxBatch = 128;

// block-grid shapes of the stage kernels
enum : int {
    kGridTiles = 0,   // (tw, th) blocks of 16 x 16: reduce, mask
    kGridDilate,      // tiles in blocks of 16 x 16: dilate
    kGridHalf,        // half-res pixels in blocks of 64 x 4
    kGridChunk,       // compaction chunks
    kGridResolve,     // queue entries (at most the half-res pixels) in blocks of 64
    kGridMip,         // half-res pixels in 8 x 8 tiles
    kGridFull,        // full-res pixels in blocks of 64 x 4
    kNumGrids
};

struct Job {
    FrameConst fc;
    Planes P;
    dof_gbuffer gb;          // as the stages read it (colour: the resolved raster plane with DOF_TAA_RASTER)
    dof_gbuffer gb_in;       // as the caller passed it
    const void *hist_in;     // nullptr when the frame has no usable history
    void *hist_out;
    uint8_t *mask;
    dof_frame_out out;
    SceneArgs scene;
    Rings grings;                 // the post-process gather's taps (lens-shaped or circular)
    uint32_t bstart[kNumGrids];   // first block of this job in each grid
    uint32_t bx[kNumGrids];       // blocks per row of this job in each grid
};

// The persistent traversal's work counters: kWorkParts slots of kWorkStride
// u32 (256 B).  Slot p holds work counter p at [0]: chunk g of a launch's rays
// (`grab` rays each) is handed out by counter g % kWorkParts, so the waves'
// takes spread over eight addresses instead of queueing on one.  From
// [kStatAt] (another 128-B line) the slot holds the statistics that the waves
// of blocks b = p mod kWorkParts add when they finish: node visits (u64),
// triangle tests (u64), stack drops (u32); a launch's totals are the sums
// over the slots.
constexpr int kWorkParts = 8, kWorkStride = 64, kStatAt = 32, kStatWords = 5;
constexpr size_t kWorkBytes = sizeof(uint32_t) * kWorkParts * kWorkStride;

struct BatchHead {      // the first 24 bytes are the batch's dof_batch_stats
    int32_t njobs;
    uint32_t rays;                       // total rays of the batch
    unsigned long long visits, tests;    // traversal statistics of the batch
    uint32_t pad[2];
    uint32_t ray_off[kMaxBatch + 1];     // first ray of each job in the batch
    alignas(8) uint32_t work[kWorkParts * kWorkStride];   // traversal work counters and statistics slots
};
static_assert(offsetof(BatchHead, visits) == 8 && offsetof(BatchHead, tests) == 16, "stats prefix");

inline size_t batch_table_bytes(int n)
{
    return (sizeof(BatchHead) + 255) / 256 * 256 + sizeof(Job) * (size_t)n;
}

// counters[] (u32) in scratch: [0] masked px, [1] rays; from [64] (256 B in)
// the traversal's work-counter and statistics slots
enum : int { kCntMasked = 0, kCntRays = 1, kCntWork = 64 };
constexpr size_t kCountersBytes = sizeof(uint32_t) * kCntWork + kWorkBytes;

// ---------------------------------------------------------------- helpers

__host__ __device__ inline float fmin_cs(float a, float b) { return b < a ? b : a; }
__host__ __device__ inline float fmax_cs(float a, float b) { return b > a ? b : a; }
__host__ __device__ inline float sat(float x) { return x > 0.0f ? (x < 1.0f ? x : 1.0f) : 0.0f; }
__host__ __device__ inline float lerp1(float a, float b, float t) { return a + (b - a) * t; }
// x clamped to [lo, hi] (lo <= hi); as max(lo, min(x, hi)) it is one med3 on the GPU
__host__ __device__ inline int clampi(int x, int lo, int hi)
{
    const int m = x < hi ? x : hi;
    return m > lo ? m : lo;
}
__host__ __device__ inline float clampf(float x, float lo, float hi) { return x < lo ? lo : (x > hi ? hi : x); }
__device__ inline float luma709(float r, float g, float b) { return (0.2126f * r + 0.7152f * g) + 0.0722f * b; }

// Full-res CoC diameter in pixels: cock * |1 - d / z| (eq. 6 solved for z).
__device__ inline float coc_px(float cock, float d, float z) { return cock * fabsf(1.0f - d / z); }

// ---------------------------------------------------------------- launchers

// api.hip: sets the calling thread's dof_last_error message and returns code
dof_status set_error(dof_status code, const char *fmt, ...);

// bvh.hip
hipError_t launch_build_bvh(SceneDev &s, hipStream_t st);

// trace.hip
int trace_blocks_per_cu(bool batch, int stack, int steps);   // resident blocks of the lens-ray traversal per CU
hipError_t launch_trace(const SceneDev &s, const FrameConst &fc, const ScratchLayout &L, char *scratch,
                        int blocks, hipStream_t st);
// the ray records of every thin-lens ray of the frame (after the compaction)
hipError_t launch_raygen(const FrameConst &fc, const ScratchLayout &L, char *scratch, hipStream_t st);
// hit record, distance, shaded colour and position of every ray (after the traversal)
// Job of a block of a batched launch: the last job whose first block in grid
// g is at or before b; (bx, by) is the block within that job's own grid.
__device__ inline int job_of_block(const Job *__restrict__ jobs, int njobs, int g, uint32_t b, uint32_t &bx,
                                   uint32_t &by)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].bstart[g] <= b) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t lb = b - jobs[lo].bstart[g], w = jobs[lo].bx[g];
    bx = lb % w;
    by = lb / w;
    return lo;
}

// ---------------------------------------------------------------- A11 resolve, shared

// One wave per 64 consecutive queue entries.  Their rays are one contiguous
// range (a pixel's rays follow each other in queue order), which the wave
// stages into LDS in chunks: fill(c0, c1, col, pos, hit) writes rays
// [c0, c1) (colour with view depth, hit position, hit id) with the 64 lanes
// sharing the work; each lane then sums its pixel's rays from LDS in ray
// order, as the single-thread loop would.
constexpr int kResolveChunk = 256;

template <class Fill>
__device__ inline void resolve_block(const FrameConst &fc, const Planes &P, const uint8_t *__restrict__ mask,
                                     const uint32_t bx, Fill fill)
{
    __shared__ float4 s_col[kResolveChunk], s_pos[kResolveChunk];
    __shared__ int32_t s_hit[kResolveChunk];
    const uint32_t masked = P.counters[kCntMasked];
    const uint32_t j0 = bx * 64;
    if (j0 >= masked) return;
    const uint32_t j = j0 + threadIdx.x;
    const bool have = j < masked;
    uint32_t q = 0, base = 0;
    int n = 0;
    if (have) {
        q = P.queue[j];
        n = mask[q];
        base = P.ray_base[j];
    }
    const uint32_t jl = min(j0 + 63u, masked - 1u);
    const uint32_t r0 = P.ray_base[j0], r1 = P.ray_base[jl] + mask[P.queue[jl]];
    float N = 0.0f, sn0 = 0.0f, sn1 = 0.0f, sn2 = 0.0f, sf0 = 0.0f, sf1 = 0.0f, sf2 = 0.0f;
    float scn = 0.0f, scf = 0.0f, fp0 = 0.0f, fp1 = 0.0f, fp2 = 0.0f, fw = 0.0f;
    for (uint32_t c0 = r0; c0 < r1; c0 += kResolveChunk) {
        const uint32_t c1 = min(c0 + (uint32_t)kResolveChunk, r1);
        fill(c0, c1, s_col, s_pos, s_hit);
        __syncthreads();
        const uint32_t kb = max(base, c0), ke = min(base + (uint32_t)n, c1);
        for (uint32_t r = kb; r < ke; ++r) {
            const float4 c = s_col[r - c0];
            const bool hit = s_hit[r - c0] >= 0;
            float w = hit ? sat(0.5f + (fc.d - c.w) / fc.ramp) : 0.0f;
            float om = 1.0f - w;
            float cz = coc_px(fc.cock, fc.d, c.w);
            N = N + w;
            sn0 = sn0 + w * c.x; sf0 = sf0 + om * c.x;
            sn1 = sn1 + w * c.y; sf1 = sf1 + om * c.y;
            sn2 = sn2 + w * c.z; sf2 = sf2 + om * c.z;
            scn = scn + w * cz;
            scf = scf + om * cz;
            if (hit) {
                const float4 p = s_pos[r - c0];
                fp0 = fp0 + om * p.x;
                fp1 = fp1 + om * p.y;
                fp2 = fp2 + om * p.z;
                fw = fw + om;
            }
        }
        __syncthreads();
    }
    if (!have) return;
    const float nf = (float)n - N;
    const bool hn = N > 0.0f, hf = nf > 0.0f, hp = fw > 0.0f;
    P.R0[q] = make_float4(hn ? sn0 / N : 0.0f, hn ? sn1 / N : 0.0f, hn ? sn2 / N : 0.0f, N);
    P.R1[q] = make_float4(hf ? sf0 / nf : 0.0f, hf ? sf1 / nf : 0.0f, hf ? sf2 / nf : 0.0f, N / (float)n);
    P.R2[q] = make_float4(hn ? scn / N : 0.0f, hf ? scf / nf : 0.0f, (float)n, 0.0f);
    P.R3[q] = make_float4(hp ? fp0 / fw : 0.0f, hp ? fp1 / fw : 0.0f, hp ? fp2 / fw : 0.0f, hp ? 1.0f : 0.0f);
}

hipError_t launch_shade_resolve(const SceneDev &s, const FrameConst &fc, const ScratchLayout &L, char *scratch,
                                const uint8_t *mask, hipStream_t st);
hipError_t launch_batch_shade_resolve(const Job *jobs, int njobs, const uint32_t *nblk, hipStream_t st);
hipError_t launch_gbuffer(const SceneDev &s, const FrameConst &fc, void *colour, int cfmt, float *depth,
                          void *normal, int nfmt, int blocks, hipStream_t st);
hipError_t launch_trace_rays(const SceneDev &s, int64_t n, const float *org, const float *dir, int32_t *hit,
                             float *t, int blocks, hipStream_t st);
// spp thin-lens rays through every full-res pixel of fc's view, chunk_px
// pixels per traversal launch; lt holds chunk_px * spp (leaf, t) records
hipError_t launch_reference(const SceneDev &s, const FrameConst &fc, int spp, uint2 *lt, int64_t chunk_px, void *colour,
                            int cfmt, int blocks, hipStream_t st);

// frame.hip
// The post-process chain (tile dilation but in the dilated mask mode,
// prefilter, gather, median, post-filter TAA) reads only what the reduce
// wrote, and only the composite reads its result: with a side stream it runs
// there, forked after the ray generation and joined before the composite,
// beside the traversal and the ray-trace stages.
struct SideStream {
    hipStream_t stream;
    hipEvent_t fork, join;   // recorded on the frame's stream / on the side stream
};
// ev (nullable): DOF_NUM_STAGES + 1 events; pre records ev[0..7], post ev[8..13]
// side (nullable, and only without ev): the post-process chain's stream
hipError_t launch_frame_pre(const FrameConst &fc, const Rings &rings, const ScratchLayout &L, char *scratch,
                            const dof_gbuffer &gb, const void *hist_in, void *hist_out, uint8_t *mask, hipEvent_t *ev,
                            const SideStream *side, hipStream_t st);
hipError_t launch_frame_post(const SceneDev &s, const FrameConst &fc, const Rings &rings, const ScratchLayout &L, char *scratch,
                             const dof_gbuffer &gb, const void *hist_in, void *hist_out, uint8_t *mask,
                             const dof_frame_out &out, hipEvent_t *ev, const SideStream *side, hipStream_t st);
hipError_t launch_history_reset(float *hist, int64_t nfloats, hipStream_t st);
// batch: head at the table start, jobs at batch_table_bytes(0); nblk[g] =
// total blocks of grid g over the jobs
// side (nullable): the post-process chain (launch_batch_chain) is left to the
// caller, to run on side->stream after the ray generation; else pre runs it
hipError_t launch_batch_pre(const BatchHead *head, const Job *jobs, int njobs, const uint32_t *nblk,
                            const Rings &rings, bool dilate, int taa, int gather_win, const SideStream *side,
                            hipStream_t st);
// the post-process chain (with_dilate: the tile dilation first)
hipError_t launch_batch_chain(const Job *jobs, int njobs, const uint32_t *nblk, const Rings &rings, bool with_dilate,
                              int taa, int gather_win, hipStream_t st);
// max_rays: the sum over the jobs of half-res pixels x m (sizes the ray generation grid)
hipError_t launch_batch_raygen(BatchHead *head, const Job *jobs, int njobs, int64_t max_rays, hipStream_t st);
hipError_t launch_batch_trace(BatchHead *head, const Job *jobs, int njobs, int blocks, const TraceKnobs &tk,
                              hipStream_t st);
// side (nullable): the composite waits for side->join
hipError_t launch_batch_post(BatchHead *head, const Job *jobs, int njobs, const uint32_t *nblk,
                             const Rings &rings, int taa, const SideStream *side, hipStream_t st);

}  // namespace dof
