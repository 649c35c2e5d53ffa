// Ray traversal kernels.
//
//  k_trace     thin-lens rays for the masked pixels (3.2.2, after Cook's
//              distributed ray tracing): persistent; each wave takes 64 ray
//              indices at a time from a device counter until the frame's ray
//              total (written by the compaction) is used up.
//  k_gbuffer   all-in-focus pinhole rays, one per full-res pixel (the sharp
//              raster image of section 3, produced by ray casting).
//  k_trace_raw closest hit of arbitrary rays.
//
// Closest hit: stack-based traversal of the binary radix tree (both child
// boxes live in the parent node, so one 64-byte fetch tests two boxes),
// watertight ray/triangle test of Woop, Benthin & Wald (JCGT 2013),
// two-sided, t > 0; equal distances resolve to the smaller triangle id, so
// the result is the same as brute force over all triangles.  The box test
// is loosened by a relative margin so that rounding can never cull a box
// holding the winning triangle.
#include "dof_internal.h"

namespace dof {
namespace {

constexpr int kTB = 128;   // threads per traversal block; LDS stack = kTB * 64 * 4 B = 32 KB

struct SceneArgs {
    int32_t ntri;
    const float4 *__restrict__ tris;
    const float4 *__restrict__ albedo;
    const BvhNode *__restrict__ nodes;
};

SceneArgs scene_args(const SceneDev &s) { return SceneArgs{s.ntri, s.tris, s.albedo, s.nodes}; }

__device__ inline float pick3(float x, float y, float z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

struct WRay {
    float o0, o1, o2;
    int kx, ky, kz;
    float sx, sy, sz;
    float ix, iy, iz;   // slab reciprocals (zero components replaced by 1e-20)
};

__device__ inline WRay make_wray(const float o[3], const float d[3])
{
    WRay r;
    r.o0 = o[0]; r.o1 = o[1]; r.o2 = o[2];
    float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    float dz = pick3(d[0], d[1], d[2], kz);
    if (dz < 0.0f) { int t = kx; kx = ky; ky = t; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.sx = pick3(d[0], d[1], d[2], kx) / dz;
    r.sy = pick3(d[0], d[1], d[2], ky) / dz;
    r.sz = 1.0f / dz;
    r.ix = 1.0f / (d[0] != 0.0f ? d[0] : 1e-20f);
    r.iy = 1.0f / (d[1] != 0.0f ? d[1] : 1e-20f);
    r.iz = 1.0f / (d[2] != 0.0f ? d[2] : 1e-20f);
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

// Conservative slab test against [0, limit]; returns entry distance.
__device__ inline bool box_hit(const WRay &r, float lx, float hx, float ly, float hy, float lz, float hz, float limit,
                               float &tenter)
{
    float t0x = (lx - r.o0) * r.ix, t1x = (hx - r.o0) * r.ix;
    float t0y = (ly - r.o1) * r.iy, t1y = (hy - r.o1) * r.iy;
    float t0z = (lz - r.o2) * r.iz, t1z = (hz - r.o2) * r.iz;
    float tn = fmax_cs(fmax_cs(fmin_cs(t0x, t1x), fmin_cs(t0y, t1y)), fmin_cs(t0z, t1z));
    float tf = fmin_cs(fmin_cs(fmax_cs(t0x, t1x), fmax_cs(t0y, t1y)), fmax_cs(t0z, t1z));
    tenter = tn;
    float slack = (fabsf(tn) + fabsf(tf)) * 9.5367431640625e-7f;   // 2^-20
    return tn <= tf + slack && tf >= -slack && tn <= limit;
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

// stack: this lane's column of the block's LDS stack (entry s at stack[s * kTB])
__device__ inline Hit closest_hit(const SceneArgs &S, const WRay &r, uint32_t *stack)
{
    Hit h{INFINITY, ~0u, 0u};
    if (S.ntri == 1) {
        consider_leaf(S, r, 0u, h);
        return h;
    }
    uint32_t node = 0;
    int sp = 0;
    while (true) {
        const BvhNode nd = S.nodes[node];
        // prune against the best hit so far, loosened by 2^-10 relative
        float limit = h.t * 1.0009765625f;
        float tl, tr;
        bool hl = box_hit(r, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.c.x, nd.c.y, limit, tl);
        bool hr = box_hit(r, nd.b.x, nd.b.y, nd.b.z, nd.b.w, nd.c.z, nd.c.w, limit, tr);
        const uint32_t L = nd.d.x, R = nd.d.y;
        if (hl && (L & kLeaf)) { consider_leaf(S, r, L & ~kLeaf, h); hl = false; }
        if (hr && (R & kLeaf)) { consider_leaf(S, r, R & ~kLeaf, h); hr = false; }
        if (hl && hr) {
            uint32_t nearc = tl <= tr ? L : R, farc = tl <= tr ? R : L;
            stack[sp * kTB] = farc;
            ++sp;
            node = nearc;
        } else if (hl) {
            node = L;
        } else if (hr) {
            node = R;
        } else {
            if (sp == 0) break;
            --sp;
            node = stack[sp * kTB];
        }
    }
    return h;
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

// Lens point by rejection from [-1, 1)^2 (24-bit lattice), at most 32 tries.
__device__ inline void lens_point(const Aperture &ap, uint32_t seed, uint32_t frame, uint32_t q, uint32_t k,
                                  float &lx, float &ly)
{
    uint32_t h = pcg_hash(pcg_hash(pcg_hash(seed) ^ frame) ^ q);
    for (uint32_t att = 0; att < 32u; ++att) {
        uint32_t a = pcg_hash(h ^ ((k << 8) | att));
        uint32_t b = pcg_hash(a);
        float x = (float)(a >> 8) * (1.0f / 8388608.0f) - 1.0f;
        float y = (float)(b >> 8) * (1.0f / 8388608.0f) - 1.0f;
        if (in_aperture(ap, x, y)) {
            lx = x;
            ly = y;
            return;
        }
    }
    lx = 0.0f;
    ly = 0.0f;
}

__device__ inline void pixel_dir(const ViewConst &v, int x, int y, int w, int h, float fv[3])
{
    float u = ((((float)x + 0.5f) * 2.0f) / (float)w - 1.0f) * v.tanx;
    float vv = (1.0f - (((float)y + 0.5f) * 2.0f) / (float)h) * v.tany;
#pragma unroll
    for (int a = 0; a < 3; ++a) fv[a] = (v.fwd[a] + u * v.right[a]) + vv * v.up[a];
}

struct TraceOut {
    const uint32_t *counters, *queue, *ray_base, *ray_pix;
    const uint8_t *mask;
    int32_t *ray_hit;
    float *ray_t;
    float4 *ray_col, *ray_pos;
    uint32_t *work;
};

__global__ __launch_bounds__(kTB) void k_trace(SceneArgs S, FrameConst fc, TraceOut T)
{
    __shared__ uint32_t stack[kStackMax * kTB];
    const int lane = threadIdx.x & 63;
    const uint32_t R = T.counters[kCntRays];
    while (true) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(T.work, 64u);
        base = __shfl(base, 0);
        if (base >= R) break;
        const uint32_t r = base + lane;
        if (r >= R) continue;
        const uint32_t j = T.ray_pix[r];
        const uint32_t q = T.queue[j];
        const uint32_t k = r - T.ray_base[j];
        const int x = (int)(q % (uint32_t)fc.hw), y = (int)(q / (uint32_t)fc.hw);
        float fv[3], pf[3], o[3], dir[3];
        pixel_dir(fc.cur, x, y, fc.hw, fc.hh, fv);
#pragma unroll
        for (int a = 0; a < 3; ++a) pf[a] = fc.cur.pos[a] + fv[a] * fc.d;
        float lx, ly;
        lens_point(fc.ap, fc.seed, fc.frame, q, k, lx, ly);
#pragma unroll
        for (int a = 0; a < 3; ++a) o[a] = fc.cur.pos[a] + fc.half_a * (lx * fc.cur.right[a] + ly * fc.cur.up[a]);
#pragma unroll
        for (int a = 0; a < 3; ++a) dir[a] = pf[a] - o[a];
        float len = sqrtf((dir[0] * dir[0] + dir[1] * dir[1]) + dir[2] * dir[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) dir[a] = dir[a] / len;
        WRay wr = make_wray(o, dir);
        Hit h = closest_hit(S, wr, stack + threadIdx.x);
        if (h.id != ~0u) {
            float P0 = o[0] + h.t * dir[0], P1 = o[1] + h.t * dir[1], P2 = o[2] + h.t * dir[2];
            float z = ((P0 - fc.cur.pos[0]) * fc.cur.fwd[0] + (P1 - fc.cur.pos[1]) * fc.cur.fwd[1]) +
                      (P2 - fc.cur.pos[2]) * fc.cur.fwd[2];
            Shaded s = shade(S, fc.shade, h.leaf, dir);
            T.ray_hit[r] = (int32_t)h.id;
            T.ray_t[r] = h.t;
            T.ray_col[r] = make_float4(s.r, s.g, s.b, z);
            T.ray_pos[r] = make_float4(P0, P1, P2, 0.0f);
        } else {
            T.ray_hit[r] = -1;
            T.ray_t[r] = INFINITY;
            T.ray_col[r] = make_float4(fc.shade.sky[0], fc.shade.sky[1], fc.shade.sky[2], INFINITY);
            T.ray_pos[r] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    }
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

__global__ __launch_bounds__(kTB) void k_gbuffer(SceneArgs S, FrameConst fc, void *colour, int cfmt, float *depth,
                                                 void *normal, int nfmt)
{
    __shared__ uint32_t stack[kStackMax * kTB];
    const int64_t p = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (p >= (int64_t)fc.W * fc.H) return;
    const int x = (int)(p % fc.W), y = (int)(p / fc.W);
    float fv[3], d[3];
    pixel_dir(fc.cur, x, y, fc.W, fc.H, fv);
    float len = sqrtf((fv[0] * fv[0] + fv[1] * fv[1]) + fv[2] * fv[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = fv[a] / len;
    WRay wr = make_wray(fc.cur.pos, d);
    Hit h = closest_hit(S, wr, stack + threadIdx.x);
    if (h.id != ~0u) {
        float P0 = fc.cur.pos[0] + h.t * d[0], P1 = fc.cur.pos[1] + h.t * d[1], P2 = fc.cur.pos[2] + h.t * d[2];
        Shaded s = shade(S, fc.shade, h.leaf, d);
        st_rgba(colour, cfmt, p, make_float4(s.r, s.g, s.b, 1.0f));
        depth[p] = ((P0 - fc.cur.pos[0]) * fc.cur.fwd[0] + (P1 - fc.cur.pos[1]) * fc.cur.fwd[1]) +
                   (P2 - fc.cur.pos[2]) * fc.cur.fwd[2];
        st_rgba(normal, nfmt, p, make_float4(s.n0, s.n1, s.n2, 0.0f));
    } else {
        st_rgba(colour, cfmt, p, make_float4(fc.shade.sky[0], fc.shade.sky[1], fc.shade.sky[2], 1.0f));
        depth[p] = INFINITY;
        st_rgba(normal, nfmt, p, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
    }
}

__global__ __launch_bounds__(kTB) void k_trace_raw(SceneArgs S, int64_t n, const float *org, const float *dir,
                                                   int32_t *hit, float *tout)
{
    __shared__ uint32_t stack[kStackMax * kTB];
    const int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (i >= n) return;
    float o[3] = {org[3 * i], org[3 * i + 1], org[3 * i + 2]};
    float d[3] = {dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
    WRay wr = make_wray(o, d);
    Hit h = closest_hit(S, wr, stack + threadIdx.x);
    hit[i] = h.id == ~0u ? -1 : (int32_t)h.id;
    tout[i] = h.t;
}

}  // namespace

hipError_t launch_trace(const SceneDev &s, const FrameConst &fc, const ScratchLayout &L, char *scratch, int blocks,
                        hipStream_t st)
{
    TraceOut T;
    T.counters = reinterpret_cast<const uint32_t *>(scratch + L.counters);
    T.work = reinterpret_cast<uint32_t *>(scratch + L.counters) + kCntWork;
    T.queue = reinterpret_cast<const uint32_t *>(scratch + L.queue);
    T.ray_base = reinterpret_cast<const uint32_t *>(scratch + L.ray_base);
    T.ray_pix = reinterpret_cast<const uint32_t *>(scratch + L.ray_pix);
    T.mask = nullptr;
    T.ray_hit = reinterpret_cast<int32_t *>(scratch + L.ray_hit);
    T.ray_t = reinterpret_cast<float *>(scratch + L.ray_t);
    T.ray_col = reinterpret_cast<float4 *>(scratch + L.ray_col);
    T.ray_pos = reinterpret_cast<float4 *>(scratch + L.ray_pos);
    k_trace<<<blocks, kTB, 0, st>>>(scene_args(s), fc, T);
    return hipGetLastError();
}

hipError_t launch_gbuffer(const SceneDev &s, const FrameConst &fc, void *colour, int cfmt, float *depth, void *normal,
                          int nfmt, hipStream_t st)
{
    int64_t n = (int64_t)fc.W * fc.H;
    k_gbuffer<<<(unsigned)((n + kTB - 1) / kTB), kTB, 0, st>>>(scene_args(s), fc, colour, cfmt, depth, normal, nfmt);
    return hipGetLastError();
}

hipError_t launch_trace_rays(const SceneDev &s, int64_t n, const float *org, const float *dir, int32_t *hit, float *t,
                             hipStream_t st)
{
    if (n == 0) return hipSuccess;
    k_trace_raw<<<(unsigned)((n + kTB - 1) / kTB), kTB, 0, st>>>(scene_args(s), n, org, dir, hit, t);
    return hipGetLastError();
}

}  // namespace dof
