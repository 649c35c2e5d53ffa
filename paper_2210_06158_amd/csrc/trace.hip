// Ray traversal kernels.
//
// One persistent kernel template serves three ray sources:
//  LensRays   thin-lens rays for the masked pixels (3.2.2, after Cook's
//             distributed ray tracing), count read from the compaction;
//  PinholeRays  all-in-focus rays, one per full-res pixel (the sharp raster
//             image of section 3, produced by ray casting);
//  RawRays    closest hit of caller-given rays.
//
// Scheduling: each lane owns one ray at a time and advances it up to three
// or four BVH nodes per loop iteration; when enough lanes of a wave are idle
// (16 by default, or all of them) the wave hands them the next rays of its
// pool, a run of 64 ray indices taken with one atomic whenever the pool is
// empty, so long rays do not hold a whole wave hostage (persistent threads
// with dynamic fetch).  The runs are dealt over eight device counters 256 B
// apart (run g by counter g mod 8), so the takes of all waves do not queue
// on one address: with a single counter they did, and a 1080p frame's
// traversal ran 10 % longer.  Thin-lens rays come from a generation kernel as
// 24-byte records (origin and direction); a lane that takes one derives the
// watertight test's shear and the slab reciprocals itself.  A finishing ray
// leaves one 8-byte (leaf, t) record that the resolve expands when it shades,
// so no lane waits on scene loads for shading.
//
// Closest hit: binary radix tree; the traversal reads a 32-byte copy of each
// node holding both children's boxes in binary16, rounded outward (one fetch
// of two 16-byte words tests two boxes).  Near child first, far child pushed
// on a per-lane stack of 16, 24 or 32 entries in LDS, so a pop is always an
// LDS read.  When the stack is full its oldest 8 entries are dropped; when it
// later runs empty the lane finds the dropped work again by walking parent
// links upwards: at each ancestor reached from its near child (entry
// distances compared as when it was first visited) whose far child still
// passes the box test, that far child is the next subtree.  Every dropped
// entry is such a far child, and the box test only loses children as the
// best hit shrinks, so the walk visits exactly the pending subtrees that can
// still hold the closest hit: any depth is exact with no memory beyond LDS.
// Each outer iteration advances a lane by up to three or four nodes (a launch
// knob), which spreads the wave-wide refill and batching decisions over
// several visits.  Leaf hits wait in a 4-entry per-lane queue and the
// triangle test runs when enough lanes of the wave have one (32 by default),
// or a queue is nearly full, or a lane has finished its traversal, so it
// executes with most lanes active instead of once per node visit for a few
// lanes; watertight ray/triangle
// test of Woop, Benthin & Wald (JCGT 2013), two-sided, t > 0, equal
// distances resolved to the smaller triangle id -- the same answer as brute
// force over all triangles.  Box tests are loosened by a relative margin so
// rounding never culls a box that holds the winning triangle.
#include "dof_internal.h"

namespace dof {
namespace {

SceneArgs scene_args(const SceneDev &s) { return SceneArgs{s.nleaf, s.tris, s.albedo, s.nodes16, s.parent}; }

__device__ inline float pick3(float x, float y, float z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

struct WRay {
    float o0, o1, o2;
    int kx, ky, kz;
    float sx, sy, sz;
    float ix, iy, iz;   // slab reciprocals (zero components replaced by 1e-20)
    float cnx, cny, cnz, cfx, cfy, cfz;   // slab offsets of the entry and exit planes (box_hit)
    uint32_t swx, swy, swz;               // 16 where the entry plane is a node word's high half, else 0
};

// The watertight test's axes: kz the largest direction component, kx and ky
// the next two in cyclic order, swapped when d[kz] < 0 (keeps the winding).
__device__ inline void wray_axes(const float d[3], int &kx, int &ky, int &kz)
{
    float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
    kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    kx = kz + 1 == 3 ? 0 : kz + 1;
    ky = kx + 1 == 3 ? 0 : kx + 1;
    if (pick3(d[0], d[1], d[2], kz) < 0.0f) { int t = kx; kx = ky; ky = t; }
}

// A plane p meets the ray at fma(p, 1/d, c) with c = -o/d.  c carries an
// absolute rounding error of at most 2^-24 |c|; it is moved outward by
// max(2^-21 |c|, 2^-30 |1/d|) (down for the entry plane, up for the exit
// plane, which one is which following the sign of 1/d), so the remaining
// errors are relative to the distance and covered by box_hit's exit margin.
// The second term widens each slab by 2^-30 in position: an axis the ray is
// parallel to (d = 0, reciprocal 1e20) then never culls a box whose slab holds
// the origin, faces included.  Needs the origin and the reciprocals; every
// construction of a WRay ends with it.
__device__ inline float slab_offset(float o, float inv, bool entry_if_positive)
{
    const float c = -(o * inv);
    const float e = fmaxf(fabsf(c) * 4.76837158203125e-07f, fabsf(inv) * 9.31322574615478515625e-10f);   // 2^-21, 2^-30
    return (inv > 0.0f) == entry_if_positive ? c - e : c + e;
}

__device__ inline void slab_offsets(WRay &r)
{
    const float clx = slab_offset(r.o0, r.ix, true), chx = slab_offset(r.o0, r.ix, false);
    const float cly = slab_offset(r.o1, r.iy, true), chy = slab_offset(r.o1, r.iy, false);
    const float clz = slab_offset(r.o2, r.iz, true), chz = slab_offset(r.o2, r.iz, false);
    const bool px = r.ix > 0.0f, py = r.iy > 0.0f, pz = r.iz > 0.0f;
    r.cnx = px ? clx : chx; r.cfx = px ? chx : clx; r.swx = px ? 0u : 16u;
    r.cny = py ? cly : chy; r.cfy = py ? chy : cly; r.swy = py ? 0u : 16u;
    r.cnz = pz ? clz : chz; r.cfz = pz ? chz : clz; r.swz = pz ? 0u : 16u;
}

__device__ inline WRay make_wray(const float o[3], const float d[3])
{
    WRay r;
    r.o0 = o[0]; r.o1 = o[1]; r.o2 = o[2];
    int kx, ky, kz;
    wray_axes(d, kx, ky, kz);
    float dz = pick3(d[0], d[1], d[2], kz);
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.sx = pick3(d[0], d[1], d[2], kx) / dz;
    r.sy = pick3(d[0], d[1], d[2], ky) / dz;
    r.sz = 1.0f / dz;
    r.ix = 1.0f / (d[0] != 0.0f ? d[0] : 1e-20f);
    r.iy = 1.0f / (d[1] != 0.0f ? d[1] : 1e-20f);
    r.iz = 1.0f / (d[2] != 0.0f ? d[2] : 1e-20f);
    slab_offsets(r);
    return r;
}

__device__ inline bool tri_hit(const WRay &r, float4 v0, float4 v1, float4 v2, float &tout)
{
    float A0 = v0.x - r.o0, A1 = v0.y - r.o1, A2 = v0.z - r.o2;
    float B0 = v1.x - r.o0, B1 = v1.y - r.o1, B2 = v1.z - r.o2;
    float C0 = v2.x - r.o0, C1 = v2.y - r.o1, C2 = v2.z - r.o2;
    float Akz = pick3(A0, A1, A2, r.kz), Bkz = pick3(B0, B1, B2, r.kz), Ckz = pick3(C0, C1, C2, r.kz);
    float Ax = pick3(A0, A1, A2, r.kx) - r.sx * Akz;
    float Ay = pick3(A0, A1, A2, r.ky) - r.sy * Akz;
    float Bx = pick3(B0, B1, B2, r.kx) - r.sx * Bkz;
    float By = pick3(B0, B1, B2, r.ky) - r.sy * Bkz;
    float Cx = pick3(C0, C1, C2, r.kx) - r.sx * Ckz;
    float Cy = pick3(C0, C1, C2, r.ky) - r.sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = U + V + W;
    if (det == 0.0f) return false;
    float Az = r.sz * Akz, Bz = r.sz * Bkz, Cz = r.sz * Ckz;
    float T = (U * Az + V * Bz) + W * Cz;
    float t = T / det;
    if (!(t > 0.0f) || !(t < INFINITY)) return false;
    tout = t;
    return true;
}

// The planes of a binary16 node word: low plane in the low half, high plane
// in the high half.  Converted exactly; the compiler folds the conversion into
// the slab test's fused multiply-add (a mixed-precision fma).
__device__ inline float lo16(uint32_t w) { return __half2float(__ushort_as_half((unsigned short)(w & 0xffffu))); }
__device__ inline float hi16(uint32_t w) { return __half2float(__ushort_as_half((unsigned short)(w >> 16))); }

// Conservative slab test of a binary16 box (three node words) against
// [0, limit]; returns the entry distance.  Each word's halves are swapped
// (alignbit by 16) where that axis' reciprocal is negative, so its low half is
// the entry plane and its high half the exit plane in every lane.  The slab
// distance is monotone in the plane (and the entry offset lies below the exit
// offset), so these are exactly the smaller and larger of the two distances:
// one swap per axis instead of a min and a max.  The test only culls, so it
// may use the hardware min/max (no NaN can arise: the reciprocals are
// finite); the exit distance is enlarged by 2^-20 relative to cover rounding.
__device__ inline bool box_hit(const WRay &r, uint32_t wx, uint32_t wy, uint32_t wz, float limit, float &tenter)
{
    wx = __builtin_amdgcn_alignbit(wx, wx, r.swx);
    wy = __builtin_amdgcn_alignbit(wy, wy, r.swy);
    wz = __builtin_amdgcn_alignbit(wz, wz, r.swz);
    float nx = fmaf(lo16(wx), r.ix, r.cnx), fx = fmaf(hi16(wx), r.ix, r.cfx);
    float ny = fmaf(lo16(wy), r.iy, r.cny), fy = fmaf(hi16(wy), r.iy, r.cfy);
    float nz = fmaf(lo16(wz), r.iz, r.cnz), fz = fmaf(hi16(wz), r.iz, r.cfz);
    float tn = fmaxf(fmaxf(nx, ny), nz);
    float tf = fminf(fminf(fx, fy), fz) * 1.00000095367431640625f;
    tenter = tn;
    // tn <= tf, tf >= 0 and tn <= limit (limit >= 0) in one comparison
    return fmaxf(tn, 0.0f) <= fminf(tf, limit);
}

// Slab tests of both children of a binary16 node.
__device__ inline void node_hits(const WRay &r, const BvhNode16 &nd, float limit, bool &hl, bool &hr, float &tl,
                                 float &tr)
{
    hl = box_hit(r, nd.a.x, nd.a.y, nd.a.z, limit, tl);
    hr = box_hit(r, nd.a.w, nd.b.x, nd.b.y, limit, tr);
}

struct Hit {
    float t;
    uint32_t id;    // original triangle id, ~0u = none
    uint32_t leaf;  // sorted position
};

__device__ inline void consider_leaf(const SceneArgs &S, const WRay &r, uint32_t leaf, Hit &h)
{
    float4 v0 = S.tris[3 * (size_t)leaf], v1 = S.tris[3 * (size_t)leaf + 1], v2 = S.tris[3 * (size_t)leaf + 2];
    float t;
    if (tri_hit(r, v0, v1, v2, t)) {
        uint32_t id = __float_as_uint(v0.w);
        if (t < h.t || (t == h.t && id < h.id)) {
            h.t = t;
            h.id = id;
            h.leaf = leaf;
        }
    }
}

struct Shaded {
    float r, g, b;
    float n0, n1, n2;
};

// Lambert: two-sided geometric normal facing the ray, one directional light
// plus ambient.
__device__ inline Shaded shade(const SceneArgs &S, const SceneShade &sh, uint32_t leaf, const float d[3])
{
    float4 v0 = S.tris[3 * (size_t)leaf], v1 = S.tris[3 * (size_t)leaf + 1], v2 = S.tris[3 * (size_t)leaf + 2];
    float e10 = v1.x - v0.x, e11 = v1.y - v0.y, e12 = v1.z - v0.z;
    float e20 = v2.x - v0.x, e21 = v2.y - v0.y, e22 = v2.z - v0.z;
    float n0 = e11 * e22 - e12 * e21, n1 = e12 * e20 - e10 * e22, n2 = e10 * e21 - e11 * e20;
    float len = sqrtf((n0 * n0 + n1 * n1) + n2 * n2);
    n0 = n0 / len; n1 = n1 / len; n2 = n2 / len;
    if ((n0 * d[0] + n1 * d[1]) + n2 * d[2] > 0.0f) { n0 = -n0; n1 = -n1; n2 = -n2; }
    float ndl = -((n0 * sh.light_dir[0] + n1 * sh.light_dir[1]) + n2 * sh.light_dir[2]);
    if (!(ndl > 0.0f)) ndl = 0.0f;
    float4 al = S.albedo[leaf];
    Shaded o;
    o.r = al.x * (sh.light_rad[0] * ndl + sh.ambient[0]);
    o.g = al.y * (sh.light_rad[1] * ndl + sh.ambient[1]);
    o.b = al.z * (sh.light_rad[2] * ndl + sh.ambient[2]);
    o.n0 = n0; o.n1 = n1; o.n2 = n2;
    return o;
}

__device__ inline uint32_t pcg_hash(uint32_t v)
{
    // PCG-RXS-M-XS hash (Jarzynski & Olano, "Hash Functions for GPU Rendering", JCGT 2020)
    uint32_t state = v * 747796405u + 2891336453u;
    uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

__device__ inline bool in_aperture(const Aperture &ap, float x, float y)
{
    if (ap.blades < 3) return x * x + y * y < 1.0f;
    for (int i = 0; i < ap.blades; ++i)
        if (x * ap.nx[i] + y * ap.ny[i] > ap.apothem) return false;
    return true;
}

// Lens point by rejection from [-1, 1)^2 (24-bit lattice), at most 32 tries:
// try att of ray k of the pixel whose hashed seed is h.
constexpr uint32_t kLensTries = 32;

__device__ inline uint32_t lens_seed(uint32_t seed, uint32_t frame, uint32_t q)
{
    return pcg_hash(pcg_hash(pcg_hash(seed) ^ frame) ^ q);
}

__device__ inline bool lens_try(const Aperture &ap, uint32_t h, uint32_t k, uint32_t att, float &x, float &y)
{
    uint32_t a = pcg_hash(h ^ ((k << 8) | att));
    uint32_t b = pcg_hash(a);
    x = (float)(a >> 8) * (1.0f / 8388608.0f) - 1.0f;
    y = (float)(b >> 8) * (1.0f / 8388608.0f) - 1.0f;
    return in_aperture(ap, x, y);
}

// The tries att0, att0 + 1, ... of a ray; (0, 0) when none of the 32 lands.
__device__ inline void lens_point_from(const Aperture &ap, uint32_t h, uint32_t k, uint32_t att0, float &lx, float &ly)
{
    for (uint32_t att = att0; att < kLensTries; ++att) {
        float x, y;
        if (lens_try(ap, h, k, att, x, y)) {
            lx = x;
            ly = y;
            return;
        }
    }
    lx = 0.0f;
    ly = 0.0f;
}

__device__ inline void lens_point(const Aperture &ap, uint32_t seed, uint32_t frame, uint32_t q, uint32_t k,
                                  float &lx, float &ly)
{
    lens_point_from(ap, lens_seed(seed, frame, q), k, 0, lx, ly);
}

__device__ inline void st_rgba(void *p, int fmt, size_t i, float4 v)
{
    if (fmt == DOF_RGBA32F) {
        reinterpret_cast<float4 *>(p)[i] = v;
    } else {
        __half2 *h = reinterpret_cast<__half2 *>(p) + 2 * i;
        h[0] = __halves2half2(__float2half(v.x), __float2half(v.y));
        h[1] = __halves2half2(__float2half(v.z), __float2half(v.w));
    }
}

// ---------------------------------------------------------------- ray sources

// Thin-lens ray k of pixel q = y w + x of a w x h grid: the pixel's point on
// the focus plane (view depth d), a lens point from the counter hash of
// (seed, frame, q, k), the normalised direction between them.
// The pixel's point on the focus plane.
__device__ inline void focus_point(const FrameConst &fc, uint32_t q, uint32_t w, uint32_t h, float pf[3])
{
    const int x = (int)(q % w), y = (int)(q / w);
    float fv[3];
    pixel_dir(fc.cur, x, y, (int)w, (int)h, fv);
#pragma unroll
    for (int a = 0; a < 3; ++a) pf[a] = fc.cur.pos[a] + fv[a] * fc.d;
}

// The ray from lens point (lx, ly) through the focus-plane point pf.
__device__ inline void lens_through(const FrameConst &fc, const float pf[3], float lx, float ly, float o[3], float d[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = fc.cur.pos[a] + fc.half_a * (lx * fc.cur.right[a] + ly * fc.cur.up[a]);
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = pf[a] - o[a];
    float len = sqrtf((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = d[a] / len;
}

__device__ inline void thin_lens_ray(const FrameConst &fc, uint32_t q, uint32_t w, uint32_t h, uint32_t k, float o[3],
                                     float d[3])
{
    float pf[3];
    focus_point(fc, q, w, h, pf);
    float lx, ly;
    lens_point(fc.ap, fc.seed, fc.frame, q, k, lx, ly);
    lens_through(fc, pf, lx, ly, o, d);
}

// Thin-lens ray r of a frame: its pixel from the ray -> pixel map, traced at
// half resolution.
__device__ inline void lens_ray(const FrameConst &fc, const uint32_t *queue, const uint32_t *ray_base,
                                const uint32_t *ray_pix, uint32_t r, float o[3], float d[3])
{
    const uint32_t j = ray_pix[r];
    thin_lens_ray(fc, queue[j], (uint32_t)fc.hw, (uint32_t)fc.hh, r - ray_base[j], o, d);
}

// Per-ray record of a lens ray: hit id, distance, shaded colour with view
// depth, hit position (sky colour and +inf depth on a miss).
// Hit id, distance, shaded colour with view depth and hit position of a lens
// ray (sky colour and +inf depth on a miss).
__device__ inline void lens_shade(const SceneArgs &S, const FrameConst &fc, const float o[3], const float d[3],
                                  const Hit &h, int32_t &hit, float &t, float4 &col, float4 &pos)
{
    if (h.id != ~0u) {
        float P0 = o[0] + h.t * d[0], P1 = o[1] + h.t * d[1], P2 = o[2] + h.t * d[2];
        float z = ((P0 - fc.cur.pos[0]) * fc.cur.fwd[0] + (P1 - fc.cur.pos[1]) * fc.cur.fwd[1]) +
                  (P2 - fc.cur.pos[2]) * fc.cur.fwd[2];
        Shaded s = dof::shade(S, fc.shade, h.leaf, d);
        hit = (int32_t)h.id;
        t = h.t;
        col = make_float4(s.r, s.g, s.b, z);
        pos = make_float4(P0, P1, P2, 0.0f);
    } else {
        hit = -1;
        t = INFINITY;
        col = make_float4(fc.shade.sky[0], fc.shade.sky[1], fc.shade.sky[2], INFINITY);
        pos = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

// Ray records (three float4 planes): (o, d.x), (d.y, d.z, sx, sy),
// (sz, 1/d.x, 1/d.y, 1/d.z), written by the ray generation kernel so that a
// traversal lane takes a new ray with three independent loads.
// A ray record is its origin and direction (24 B: a float4 and a float2
// plane); the traversal derives the watertight shear and the reciprocals when
// a lane takes the ray (six correctly rounded divides, shared by the lanes a
// refill starts), which costs less than moving them through memory.
__device__ inline void put_ray(float4 *rec0, float2 *rec1, uint32_t r, const float o[3], const float d[3])
{
    rec0[r] = make_float4(o[0], o[1], o[2], d[0]);
    rec1[r] = make_float2(d[1], d[2]);
}

__device__ inline void get_ray(const float4 *rec0, const float2 *rec1, uint32_t r, float o[3], float d[3], WRay &w)
{
    const float4 a = rec0[r];
    const float2 b = rec1[r];
    o[0] = a.x; o[1] = a.y; o[2] = a.z;
    d[0] = a.w; d[1] = b.x; d[2] = b.y;
    w = make_wray(o, d);
}

// The traversal's result of a lens ray: leaf of the closest hit (~0u: none)
// and distance, one 8-byte store; the resolve expands it when it shades.
__device__ inline void put_lt(uint2 *lt, uint32_t r, const Hit &h)
{
    lt[r] = make_uint2(h.id == ~0u ? ~0u : h.leaf, __float_as_uint(h.t));
}

// Origin, direction and closest hit of lens ray r, from its ray record and
// its traversal result.
__device__ inline void ray_of(const SceneArgs &S, const Planes &P, uint32_t r, float o[3], float d[3], Hit &h)
{
    const uint2 lt = P.ray_lt[r];
    const float4 a = P.rec0[r];
    const float2 b = P.rec1[r];
    o[0] = a.x; o[1] = a.y; o[2] = a.z;
    d[0] = a.w; d[1] = b.x; d[2] = b.y;
    h.t = __uint_as_float(lt.y);
    h.leaf = lt.x;
    h.id = lt.x == ~0u ? ~0u : __float_as_uint(S.tris[3 * (size_t)lt.x].w);
}

struct LensRays {
    static constexpr bool kPerLaneScene = false;
    const float4 *rec0;
    const float2 *rec1;
    uint2 *ray_lt;

    __device__ void start(uint32_t r, float o[3], float d[3], WRay &w) const { get_ray(rec0, rec1, r, o, d, w); }

    __device__ void finish(const SceneArgs &, uint32_t r, const float *, const float *, const Hit &h) const
    {
        put_lt(ray_lt, r, h);
    }
};

// Lens rays of all frames of a batch: ray r belongs to the last job whose
// first ray is at or before r (found in an LDS copy of the jobs' first rays);
// each lane remembers its ray's job and traces against that job's scene.
struct BatchRays {
    static constexpr bool kPerLaneScene = true;
    const Job *jobs;
    const BatchHead *head;
    int njobs;

    __device__ static uint32_t *offsets()
    {
        __shared__ uint32_t off[kMaxBatch + 1];
        return off;
    }

    __device__ void init() const
    {
        uint32_t *off = offsets();
        for (int j = threadIdx.x; j <= njobs; j += blockDim.x) off[j] = head->ray_off[j];
        __syncthreads();
    }

    __device__ int job_of(uint32_t r) const
    {
        const uint32_t *off = offsets();
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= r) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }

    __device__ SceneArgs scene(int j) const { return jobs[j].scene; }

    __device__ void start(uint32_t r, int j, float o[3], float d[3], WRay &w) const
    {
        const Job &J = jobs[j];
        get_ray(J.P.rec0, J.P.rec1, r - offsets()[j], o, d, w);
    }

    __device__ void finish(const SceneArgs &, uint32_t r, int j, const float *, const float *, const Hit &h) const
    {
        put_lt(jobs[j].P.ray_lt, r - offsets()[j], h);
    }
};

struct PinholeRays {
    static constexpr bool kPerLaneScene = false;
    FrameConst fc;
    SceneShade shade;
    void *colour;
    int cfmt;
    float *depth;
    void *normal;
    int nfmt;

    __device__ void start(uint32_t p, float o[3], float d[3], WRay &w) const
    {
        setup(p, o, d);
        w = make_wray(o, d);
    }

    __device__ void setup(uint32_t p, float o[3], float d[3]) const
    {
        const int x = (int)(p % (uint32_t)fc.W), y = (int)(p / (uint32_t)fc.W);
        float fv[3];
        pixel_dir(fc.cur, x, y, fc.W, fc.H, fv);
        float len = sqrtf((fv[0] * fv[0] + fv[1] * fv[1]) + fv[2] * fv[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            d[a] = fv[a] / len;
            o[a] = fc.cur.pos[a];
        }
    }

    __device__ void finish(const SceneArgs &S, uint32_t p, const float o[3], const float d[3], const Hit &h) const
    {
        if (h.id != ~0u) {
            float P0 = o[0] + h.t * d[0], P1 = o[1] + h.t * d[1], P2 = o[2] + h.t * d[2];
            Shaded s = dof::shade(S, shade, h.leaf, d);
            st_rgba(colour, cfmt, p, make_float4(s.r, s.g, s.b, 1.0f));
            depth[p] = ((P0 - fc.cur.pos[0]) * fc.cur.fwd[0] + (P1 - fc.cur.pos[1]) * fc.cur.fwd[1]) +
                       (P2 - fc.cur.pos[2]) * fc.cur.fwd[2];
            st_rgba(normal, nfmt, p, make_float4(s.n0, s.n1, s.n2, 0.0f));
        } else {
            st_rgba(colour, cfmt, p, make_float4(shade.sky[0], shade.sky[1], shade.sky[2], 1.0f));
            depth[p] = INFINITY;
            st_rgba(normal, nfmt, p, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
        }
    }
};

struct RawRays {
    static constexpr bool kPerLaneScene = false;
    const float *org, *dir;
    int32_t *hit;
    float *t;

    __device__ void start(uint32_t i, float o[3], float d[3], WRay &w) const
    {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = org[3 * (size_t)i + a];
            d[a] = dir[3 * (size_t)i + a];
        }
        w = make_wray(o, d);
    }

    __device__ void finish(const SceneArgs &, uint32_t i, const float *, const float *, const Hit &h) const
    {
        hit[i] = h.id == ~0u ? -1 : (int32_t)h.id;
        t[i] = h.t;
    }
};

// The fully ray-traced image (ground truth of the accuracy judge): ray r of
// a chunk is sample k = r mod spp of full-res pixel p0 + r / spp, traced at
// full resolution with the frame's lens; its (leaf, t) result goes to lt[r].
struct RefRays {
    static constexpr bool kPerLaneScene = false;
    FrameConst fc;
    uint32_t p0, spp;
    uint2 *lt;

    __device__ void ray(uint32_t r, float o[3], float d[3]) const
    {
        thin_lens_ray(fc, p0 + r / spp, (uint32_t)fc.W, (uint32_t)fc.H, r % spp, o, d);
    }

    __device__ void start(uint32_t r, float o[3], float d[3], WRay &w) const
    {
        ray(r, o, d);
        w = make_wray(o, d);
    }

    __device__ void finish(const SceneArgs &, uint32_t r, const float *, const float *, const Hit &h) const
    {
        put_lt(lt, r, h);
    }
};

// Mean shaded colour of each pixel's spp rays of a chunk (binary64 sum in
// sample order, one rounding to binary32).
__global__ __launch_bounds__(256) void k_ref_average(SceneArgs S, RefRays src, uint32_t npx, void *colour, int cfmt)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= npx) return;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    for (uint32_t k = 0; k < src.spp; ++k) {
        const uint32_t r = i * src.spp + k;
        float o[3], d[3];
        src.ray(r, o, d);
        const uint2 lt = src.lt[r];
        Hit h;
        h.t = __uint_as_float(lt.y);
        h.leaf = lt.x;
        h.id = lt.x == ~0u ? ~0u : __float_as_uint(S.tris[3 * (size_t)lt.x].w);
        int32_t hi;
        float t;
        float4 c, p;
        lens_shade(S, src.fc, o, d, h, hi, t, c, p);
        acc0 += (double)c.x;
        acc1 += (double)c.y;
        acc2 += (double)c.z;
    }
    const double n = (double)src.spp;
    st_rgba(colour, cfmt, (size_t)src.p0 + i, make_float4((float)(acc0 / n), (float)(acc1 / n), (float)(acc2 / n), 1.0f));
}

// ---------------------------------------------------------------- ray generation

constexpr int kGenTB = 256;
constexpr int kGenMaxBlocks = 2048;

// Every thin-lens ray of a frame (the count is the compaction's ray total).
__global__ __launch_bounds__(kGenTB) void k_raygen(FrameConst fc, const uint32_t *queue, const uint32_t *ray_base,
                                                   const uint32_t *ray_pix, const uint32_t *count, float4 *rec0,
                                                   float2 *rec1)
{
    const uint32_t N = *count;
    for (uint32_t r = blockIdx.x * kGenTB + threadIdx.x; r < N; r += gridDim.x * kGenTB) {
        float o[3], d[3];
        lens_ray(fc, queue, ray_base, ray_pix, r, o, d);
        put_ray(rec0, rec1, r, o, d);
    }
}

// The same for a bladed aperture, whose lens points take more tries
// (rejection from the square keeps 65 % of them for a hexagon against 79 %
// for a circle).  A wave walks runs of up to kGenSpan rays (shorter when the
// frame has few rays, so every wave gets some); each ray first gets
// kGenFirst tries, the rays still without a point wait in a per-wave LDS
// list, and the wave then runs the remaining tries for them one per lane, so
// it does not spin for its unluckiest lane while the others idle.  Every ray
// gets the same tries in the same order as one lens_point call.
constexpr int kGenSpan = 512;
constexpr uint32_t kGenFirst = 2;

__global__ __launch_bounds__(kGenTB) void k_raygen_bladed(FrameConst fc, const uint32_t *queue,
                                                          const uint32_t *ray_base, const uint32_t *ray_pix,
                                                          const uint32_t *count, float4 *rec0, float2 *rec1)
{
    __shared__ uint32_t left[kGenTB / 64][kGenSpan];
    const uint32_t N = *count;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t nwaves = gridDim.x * (kGenTB / 64);
    const uint32_t hw = (uint32_t)fc.hw, hh = (uint32_t)fc.hh;
    uint32_t span = ((N / nwaves + 1u) + 63u) & ~63u;
    span = span < (uint32_t)kGenSpan ? span : (uint32_t)kGenSpan;
    for (uint32_t base = (blockIdx.x * (kGenTB / 64) + w) * span; base < N; base += nwaves * span) {
        const uint32_t end = N - base < span ? N : base + span;
        uint32_t nleft = 0;   // wave-uniform
        for (uint32_t r0 = base; r0 < end; r0 += 64) {
            const uint32_t r = r0 + (uint32_t)lane;
            bool miss = false;
            if (r < end) {
                const uint32_t j = ray_pix[r], q = queue[j], k = r - ray_base[j];
                const uint32_t hs = lens_seed(fc.seed, fc.frame, q);
                float lx = 0.0f, ly = 0.0f;
                bool ok = false;
                for (uint32_t att = 0; att < kGenFirst && !ok; ++att) ok = lens_try(fc.ap, hs, k, att, lx, ly);
                if (ok) {
                    float pf[3], o[3], d[3];
                    focus_point(fc, q, hw, hh, pf);
                    lens_through(fc, pf, lx, ly, o, d);
                    put_ray(rec0, rec1, r, o, d);
                } else {
                    miss = true;
                }
            }
            const uint64_t m = __ballot(miss);
            if (miss) left[w][nleft + (uint32_t)__popcll(m & lt)] = r;
            nleft += (uint32_t)__popcll(m);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t t = (uint32_t)lane; t < nleft; t += 64) {
            const uint32_t r = left[w][t];
            const uint32_t j = ray_pix[r], q = queue[j], k = r - ray_base[j];
            float lx, ly, pf[3], o[3], d[3];
            lens_point_from(fc.ap, lens_seed(fc.seed, fc.frame, q), k, kGenFirst, lx, ly);
            focus_point(fc, q, hw, hh, pf);
            lens_through(fc, pf, lx, ly, o, d);
            put_ray(rec0, rec1, r, o, d);
        }
        __builtin_amdgcn_wave_barrier();   // the list is rewritten by the next run
    }
}

__global__ __launch_bounds__(kGenTB) void kb_raygen(const Job *__restrict__ jobs, const BatchHead *head, int njobs)
{
    __shared__ uint32_t off[kMaxBatch + 1];
    for (int j = threadIdx.x; j <= njobs; j += kGenTB) off[j] = head->ray_off[j];
    __syncthreads();
    const uint32_t N = head->rays;
    for (uint32_t r = blockIdx.x * kGenTB + threadIdx.x; r < N; r += gridDim.x * kGenTB) {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= r) lo = mid;
            else hi = mid - 1;
        }
        const Job &J = jobs[lo];
        const uint32_t k = r - off[lo];
        float o[3], d[3];
        lens_ray(J.fc, J.P.queue, J.P.ray_base, J.P.ray_pix, k, o, d);
        put_ray(J.P.rec0, J.P.rec1, k, o, d);
    }
}

// Shading and resolve of a frame's lens rays in one pass: each block shades
// the rays of its 64 pixels straight into the resolve's LDS chunks (and, when
// the frame keeps them, into the per-ray planes), so nothing is read back.
__device__ inline void shade_resolve_block(const SceneArgs &S, const FrameConst &fc, const Planes &P,
                                           const uint8_t *__restrict__ mask, uint32_t bx)
{
    resolve_block(fc, P, mask, bx, [&](uint32_t c0, uint32_t c1, float4 *col, float4 *pos, int32_t *hit) {
        for (uint32_t r = c0 + threadIdx.x; r < c1; r += 64) {
            float o[3], d[3];
            Hit h;
            ray_of(S, P, r, o, d, h);
            int32_t hi;
            float t;
            float4 c, p;
            lens_shade(S, fc, o, d, h, hi, t, c, p);
            if (P.ray_hit) {   // per-ray planes kept for inspection (params.ray_records)
                P.ray_hit[r] = hi;
                P.ray_t[r] = t;
                P.ray_col[r] = c;
                P.ray_pos[r] = p;
            }
            col[r - c0] = c;
            pos[r - c0] = p;
            hit[r - c0] = hi;
        }
    });
}

__global__ __launch_bounds__(64) void k_shade_resolve(SceneArgs S, FrameConst fc, Planes P,
                                                      const uint8_t *__restrict__ mask)
{
    shade_resolve_block(S, fc, P, mask, blockIdx.x);
}

__global__ __launch_bounds__(64) void kb_shade_resolve(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridResolve, blockIdx.x, bx, by)];
    shade_resolve_block(J.scene, J.fc, J.P, J.mask, bx);
}

int gen_blocks(int64_t max_rays)
{
    const int64_t b = (max_rays + kGenTB - 1) / kGenTB;
    return b < 1 ? 1 : (b > kGenMaxBlocks ? kGenMaxBlocks : (int)b);
}

// ---------------------------------------------------------------- persistent traversal

constexpr int kDropChunk = 8;    // oldest stack entries dropped when the LDS stack is full
// Launch knobs (TraceKnobs, defaults in brackets): a wave refills when at
// least tk.refill lanes are idle [16], takes tk.grab rays from the work
// counters at a time [64], and runs its triangle tests when at least
// tk.leaf_batch lanes have one pending [32]; kStack LDS stack entries per
// lane [24]; kSteps node visits per lane per iteration [4]; tk.reverse
// hands the rays out from the end of the queue [for
// frames; the scene-level sources keep the queue order].  The last rays a
// persistent grid hands out set its tail: when they are cheap, every wave
// finishes at nearly the same time.

// work: slot 0 of the work-counter slots; stats and drops_out (or null):
// slot 0's node-visit and stack-drop statistics, a wave adding its totals to
// the slot of its block (b mod kWorkParts) when it finishes.
// Occupancy: at 77 VGPRs a lane, six waves fit a SIMD; with the 16-entry
// stack the LDS would hold ten, and asking for seven (72 VGPRs, two spilled)
// lets 14 instead of 12 blocks share a compute unit -- 4 % less traversal
// time at 3840x2160, the same at 1920x1080.  A batch's lanes also hold their
// scene's pointers (84 VGPRs: five waves); asking for six (80, none spilled)
// makes a 32-session batch 3.6 % faster.  The 32-entry stack is LDS-bound
// below both.
template <class Src, int kStack, int kSteps>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(Src::kPerLaneScene ? (kStack == 32 ? 1 : 6) : (kStack == 16 ? 7 : 1))))
void k_traverse(SceneArgs S, Src src, uint32_t count, const uint32_t *count_ptr,
                                                  uint32_t *work, unsigned long long *stats, uint32_t *drops_out,
                                                  TraceKnobs tk)
{
    static_assert(kDropChunk < kStack, "a drop must leave room for the push");
    __shared__ uint32_t lds_stack[kStack * kTB];
    const uint32_t grab = tk.grab;
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t N = count_ptr ? *count_ptr : count;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t *stk = lds_stack + tid;

    bool active = false, exhausted = false;
    // rays [pool, pool_end) taken by this wave and not yet handed to a lane
    // (wave-uniform); a new batch of `grab` comes from the work counters only
    // when the pool is empty, so refills rarely touch an atomic
    uint32_t pool = 0, pool_end = 0;
    bool drained = false;   // every work counter has passed N (wave-uniform)
    uint32_t part = blockIdx.x % kWorkParts;   // the work counter this wave takes from first
    uint32_t item = 0, node = 0;
    int sp = 0;             // entries on the LDS stack
    bool dropped = false;   // entries of this ray were dropped (found again through parent links)
    float o[3], d[3];
    WRay wr;
    Hit h;
    uint32_t visits = 0, tests = 0, drops = 0;
    // pending leaf hits of this lane (tested when enough lanes have some)
    uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0;
    int nq = 0;
    bool trav = false;   // the lane still has an inner node to visit
    SceneArgs Sl = S;    // scene of the lane's ray (differs per lane in a batch)
    int job = 0;         // job of the lane's ray (batches)
    if constexpr (Src::kPerLaneScene) src.init();

    while (true) {
        const uint64_t idle = __ballot(!active && !exhausted);
        const uint64_t live = __ballot(active);
        if (idle != 0ull && (__popcll(idle) >= tk.refill || live == 0ull)) {
            if (pool == pool_end && !drained) {
                // chunk g = k * kWorkParts + part is the k-th take of counter
                // part; a counter past the last chunk sends the wave on to
                // the next, and a wave that finds all past it is drained
                uint32_t base = N;
                if (lane == 0) {
                    for (int t = 0; t < kWorkParts; ++t) {
                        const uint32_t k = atomicAdd(work + part * kWorkStride, 1u);
                        const uint64_t b = ((uint64_t)k * kWorkParts + part) * grab;
                        if (b < N) {
                            base = (uint32_t)b;
                            break;
                        }
                        part = part + 1 == kWorkParts ? 0u : part + 1;
                    }
                }
                base = __shfl(base, 0);
                part = __shfl(part, 0);
                if (base >= N) {
                    drained = true;
                } else {
                    pool = base;
                    pool_end = N - base < grab ? N : base + grab;
                }
            }
            const uint32_t avail = pool_end - pool;
            const uint32_t rank = (uint32_t)__popcll(idle & lt);
            if (!active && !exhausted) {
                item = pool + rank;
                if (rank < avail) {
                    if (tk.reverse) item = N - 1u - item;   // pool + rank < N
                    if constexpr (Src::kPerLaneScene) {
                        job = src.job_of(item);
                        Sl = src.scene(job);
                        src.start(item, job, o, d, wr);
                    } else {
                        src.start(item, o, d, wr);
                    }
                    h = Hit{INFINITY, ~0u, 0u};
                    node = 0;
                    sp = 0;
                    dropped = false;
                    nq = 0;
                    active = true;
                    if (Sl.nleaf == 1) {
                        trav = false;
                        q0 = 0u;
                        nq = 1;
                    } else {
                        trav = true;
                    }
                } else if (drained) {
                    exhausted = true;
                }
            }
            const uint32_t nidle = (uint32_t)__popcll(idle);
            pool += nidle < avail ? nidle : avail;
        }
        if (__ballot(active) == 0ull) {
            if (__ballot(!exhausted) == 0ull) break;
            continue;
        }
        // triangle tests, batched across the wave
        const bool want = active && nq > 0;
        const bool must = want && (nq >= 3 || !trav);
        if (__ballot(must) != 0ull || __popcll(__ballot(want)) >= tk.leaf_batch) {
            if (want) {
                ++tests;
                consider_leaf(Sl, wr, q0, h);
                q0 = q1; q1 = q2; q2 = q3;
                --nq;
            }
        }
#pragma unroll
        for (int step = 0; step < kSteps; ++step) {
            if (!(active && trav && nq <= 2)) continue;
            const uint32_t nd_self = node;
            const BvhNode16 nd = Sl.nodes[node];
            ++visits;
            const float limit = h.t * 1.0009765625f;   // prune against the best hit, 2^-10 relative slack
            float tl, tr;
            bool hl, hr;
            node_hits(wr, nd, limit, hl, hr, tl, tr);
            const uint32_t L = nd.b.z, R = nd.b.w;
            // leaf children go to the front of the pending queue (shift in)
            const bool pl = hl && (L & kLeaf) != 0u, pr = hr && (R & kLeaf) != 0u;
            q3 = pl ? q2 : q3; q2 = pl ? q1 : q2; q1 = pl ? q0 : q1; q0 = pl ? (L & ~kLeaf) : q0;
            q3 = pr ? q2 : q3; q2 = pr ? q1 : q2; q1 = pr ? q0 : q1; q0 = pr ? (R & ~kLeaf) : q0;
            nq += (int)pl + (int)pr;
            hl = hl && !pl;
            hr = hr && !pr;
            const bool both = hl && hr;
            const bool none = !hl && !hr;
            if (both && sp == kStack) {
                // stack full: the oldest entries go (the parent walk finds them again)
                for (int i = 0; i < kStack - kDropChunk; ++i) stk[i * kTB] = stk[(i + kDropChunk) * kTB];
                sp -= kDropChunk;
                dropped = true;
                ++drops;
            }
            // next node by selects (no divergent branches): the near child when both are
            // hit (the far one pushed), else the one hit child, else the stack top
            const bool nearl = tl <= tr;
            if (both) stk[sp * kTB] = nearl ? R : L;
            const bool pop = none && sp > 0;
            uint32_t top = 0u;
            if (pop) top = stk[(sp - 1) * kTB];
            const uint32_t one = hl ? L : R;
            node = both ? (nearl ? L : R) : (none ? top : one);
            sp += both ? 1 : (pop ? -1 : 0);
            if (none && !pop) {
                trav = false;
                if (dropped) {
                    // stack empty after a drop: walk up from this finished subtree
                    // to the nearest ancestor whose far child is still pending
                    uint32_t c = nd_self;
                    for (uint32_t a = Sl.parent[c]; a != ~0u; c = a, a = Sl.parent[a]) {
                        const BvhNode16 pn = Sl.nodes[a];
                        ++visits;
                        const float lim = h.t * 1.0009765625f;
                        float ta, tb;
                        bool ha, hb;
                        node_hits(wr, pn, lim, ha, hb, ta, tb);
                        const bool from_left = pn.b.z == c;
                        const uint32_t other = from_left ? pn.b.w : pn.b.z;
                        const bool came_near = from_left ? ta <= tb : !(ta <= tb);
                        if (came_near && (other & kLeaf) == 0u && (from_left ? hb : ha)) {
                            node = other;
                            trav = true;
                            break;
                        }
                    }
                }
            }
        }
        if (active && !trav && nq == 0) {
            if constexpr (Src::kPerLaneScene) src.finish(Sl, item, job, o, d, h);
            else src.finish(Sl, item, o, d, h);
            active = false;
        }
    }
    if (stats) {
        unsigned long long v = visits, t = tests;
        for (int off = 32; off >= 1; off >>= 1) {
            v += __shfl_xor(v, off);
            t += __shfl_xor(t, off);
        }
        if (lane == 0) {
            unsigned long long *slot = stats + (blockIdx.x % kWorkParts) * (kWorkStride / 2);
            atomicAdd(slot, v);
            atomicAdd(slot + 1, t);
        }
    }
    if (drops_out) {
        uint32_t sv = drops;
        for (int off = 32; off >= 1; off >>= 1) sv += __shfl_xor(sv, off);
        if (lane == 0 && sv) atomicAdd(drops_out + (blockIdx.x % kWorkParts) * kWorkStride, sv);
    }
}

__global__ void k_zero_work(uint32_t *work)
{
    if ((int)threadIdx.x < kWorkParts) work[threadIdx.x * kWorkStride] = 0u;
}

// First ray of every job of a batch (exclusive prefix of the jobs' ray
// counts), the batch total, and cleared traversal counters.
__global__ void kb_ray_offsets(BatchHead *head, const Job *__restrict__ jobs, int njobs)
{
    if (threadIdx.x != 0) return;
    uint32_t acc = 0;
    for (int j = 0; j < njobs; ++j) {
        head->ray_off[j] = acc;
        acc += jobs[j].P.counters[kCntRays];
    }
    head->ray_off[njobs] = acc;
    head->rays = acc;
    for (int p = 0; p < kWorkParts; ++p) {
        uint32_t *w = head->work + p * kWorkStride;
        w[0] = 0u;
        for (int k = 0; k < kStatWords; ++k) w[kStatAt + k] = 0u;
    }
    head->visits = 0ull;
    head->tests = 0ull;
}

int clamp_blocks(int blocks) { return blocks < 1 ? 1 : (blocks > kMaxTraceBlocks ? kMaxTraceBlocks : blocks); }

}  // namespace

// The traversal kernel of a ray source for a stack depth and a number of
// node visits per loop iteration: f(kernel).
template <class Src, int kStack, class F>
void with_steps(int steps, F f)
{
    if (steps == 3) f(k_traverse<Src, kStack, 3>);
    else f(k_traverse<Src, kStack, 4>);
}

template <class Src, class F>
void with_shape(int stack, int steps, F f)
{
    if (stack == 16) with_steps<Src, 16>(steps, f);
    else if (stack == 32) with_steps<Src, 32>(steps, f);
    else with_steps<Src, kStackLds>(steps, f);
}

int trace_blocks_per_cu(bool batch, int stack, int steps)
{
    int n = 0;
    hipError_t e = hipSuccess;
    auto occ = [&](auto kern) { e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kTB, 0); };
    if (batch) with_shape<BatchRays>(stack, steps, occ);
    else with_shape<LensRays>(stack, steps, occ);
    return e == hipSuccess ? n : 0;
}

hipError_t launch_trace(const SceneDev &s, const FrameConst &fc, const ScratchLayout &L, char *scratch, int blocks,
                        hipStream_t st)
{
    LensRays src;
    const Planes P = planes(fc, L, scratch);
    src.rec0 = P.rec0;
    src.rec1 = P.rec1;
    src.ray_lt = P.ray_lt;
    uint32_t *cnt = reinterpret_cast<uint32_t *>(scratch + L.counters);
    with_shape<LensRays>(fc.tk.stack, fc.tk.steps, [&](auto kern) {
        kern<<<clamp_blocks(blocks), kTB, 0, st>>>(scene_args(s), src, 0u, cnt + kCntRays, cnt + kCntWork,
                                                  reinterpret_cast<unsigned long long *>(cnt + kCntWork + kStatAt),
                                                  cnt + kCntWork + kStatAt + 4, fc.tk);
    });
    return hipGetLastError();
}

hipError_t launch_raygen(const FrameConst &fc, const ScratchLayout &L, char *scratch, hipStream_t st)
{
    const Planes P = planes(fc, L, scratch);
    const int64_t max_rays = (int64_t)fc.hw * fc.hh * fc.m;
    if (fc.ap.blades >= 3)
        k_raygen_bladed<<<gen_blocks(max_rays), kGenTB, 0, st>>>(fc, P.queue, P.ray_base, P.ray_pix,
                                                                 P.counters + kCntRays, P.rec0, P.rec1);
    else
        k_raygen<<<gen_blocks(max_rays), kGenTB, 0, st>>>(fc, P.queue, P.ray_base, P.ray_pix, P.counters + kCntRays,
                                                           P.rec0, P.rec1);
    return hipGetLastError();
}

hipError_t launch_batch_shade_resolve(const Job *jobs, int njobs, const uint32_t *nblk, hipStream_t st)
{
    kb_shade_resolve<<<nblk[kGridResolve], 64, 0, st>>>(jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_shade_resolve(const SceneDev &s, const FrameConst &fc, const ScratchLayout &L, char *scratch,
                                const uint8_t *mask, hipStream_t st)
{
    const Planes P = planes(fc, L, scratch);
    const int64_t np = (int64_t)fc.hw * fc.hh;
    k_shade_resolve<<<(unsigned)((np + 63) / 64), 64, 0, st>>>(scene_args(s), fc, P, mask);
    return hipGetLastError();
}

hipError_t launch_gbuffer(const SceneDev &s, const FrameConst &fc, void *colour, int cfmt, float *depth, void *normal,
                          int nfmt, int blocks, hipStream_t st)
{
    PinholeRays src;
    src.fc = fc;
    src.shade = fc.shade;
    src.colour = colour;
    src.cfmt = cfmt;
    src.depth = depth;
    src.normal = normal;
    src.nfmt = nfmt;
    k_zero_work<<<1, 64, 0, st>>>(s.aux);
    k_traverse<PinholeRays, kStackLds, kTraceSteps><<<clamp_blocks(blocks), kTB, 0, st>>>(
        scene_args(s), src, (uint32_t)((int64_t)fc.W * fc.H), nullptr, s.aux, nullptr, nullptr, fc.tk);
    return hipGetLastError();
}

hipError_t launch_trace_rays(const SceneDev &s, int64_t n, const float *org, const float *dir, int32_t *hit, float *t,
                             int blocks, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    RawRays src{org, dir, hit, t};
    k_zero_work<<<1, 64, 0, st>>>(s.aux);
    TraceKnobs tk{kStackLds, 64u, 16, 32};
    k_traverse<RawRays, kStackLds, kTraceSteps><<<clamp_blocks(blocks), kTB, 0, st>>>(scene_args(s), src, (uint32_t)n, nullptr, s.aux,
                                                                         nullptr, nullptr, tk);
    return hipGetLastError();
}

hipError_t launch_reference(const SceneDev &s, const FrameConst &fc, int spp, uint2 *lt, int64_t chunk_px, void *colour,
                            int cfmt, int blocks, hipStream_t st)
{
    const int64_t npx = (int64_t)fc.W * fc.H;
    for (int64_t p0 = 0; p0 < npx; p0 += chunk_px) {
        const uint32_t n = (uint32_t)(npx - p0 < chunk_px ? npx - p0 : chunk_px);
        RefRays src{fc, (uint32_t)p0, (uint32_t)spp, lt};
        k_zero_work<<<1, 64, 0, st>>>(s.aux);
        k_traverse<RefRays, kStackLds, kTraceSteps><<<clamp_blocks(blocks), kTB, 0, st>>>(scene_args(s), src, n * (uint32_t)spp,
                                                                            nullptr, s.aux, nullptr, nullptr, fc.tk);
        k_ref_average<<<(n + 255) / 256, 256, 0, st>>>(scene_args(s), src, n, colour, cfmt);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batch_raygen(BatchHead *head, const Job *jobs, int njobs, int64_t max_rays, hipStream_t st)
{
    kb_ray_offsets<<<1, 64, 0, st>>>(head, jobs, njobs);
    kb_raygen<<<gen_blocks(max_rays), kGenTB, 0, st>>>(jobs, head, njobs);
    return hipGetLastError();
}

hipError_t launch_batch_trace(BatchHead *head, const Job *jobs, int njobs, int blocks, const TraceKnobs &tk,
                              hipStream_t st)
{
    BatchRays src{jobs, head, njobs};
    with_shape<BatchRays>(tk.stack, tk.steps, [&](auto kern) {
        kern<<<clamp_blocks(blocks), kTB, 0, st>>>(SceneArgs{}, src, 0u, &head->rays, head->work,
                                                  reinterpret_cast<unsigned long long *>(head->work + kStatAt),
                                                  nullptr, tk);
    });
    return hipGetLastError();
}

}  // namespace dof
