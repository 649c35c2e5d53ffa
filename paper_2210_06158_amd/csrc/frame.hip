// Per-frame kernels of the hybrid depth-of-field pass, except the ray
// traversal (trace.hip).  Stage names follow section 3 of the paper:
//   A1  CoC + half-res reduce (+ per-tile max CoC)          3.1, 3.3 eq. 6
//   A2  tile-neighbourhood max CoC                          3.1.1
//   A3  9-tap bilateral prefilter                           3.1.1
//   A4  81-tap near/far gather, eq. (1)                     3.1.2
//   A5  3x3 median postfilter                               3.1.3
//   A6  ray mask, eqs. (2)-(4)                              3.2.1
//   A7  ordered compaction of masked pixels into a queue    (GPU dispatch)
//   A11 near/far resolve and hit ratio                      3.2.2
//   A12 temporal accumulation, reprojection, variance       3.2.3
//   A13 median, mip chain, spatial reconstruction, eq. (5)(8)  3.2.4
//   A14 composite, eqs. (6)(7)                              3.3
// Every floating-point expression is evaluated in the order written, in
// binary32 without contraction, so that index decisions (nearest texels,
// ray counts) are reproducible.
#include "dof_internal.h"

namespace dof {
namespace {

constexpr int kBX = 64, kBY = 4;   // pixel-kernel block: one wave per row

// The dispatcher deals workgroups round-robin to the 8 XCDs (workgroup i to
// XCD i mod 8), each with its own L2.  xcd_tile renumbers the tiles of a 2-D
// grid so that XCD x takes one contiguous run of them in row-major order:
// neighbouring tiles, whose tap footprints overlap, then share one L2 instead
// of fetching the same halo into several.  A bijection for any grid size, so
// only the order of the work changes.  Worth it for the wide, uniform-cost
// gather; kernels whose cost follows the ray mask keep the interleaved order,
// which spreads expensive regions over all XCDs.
__device__ inline void xcd_tile(uint32_t &bx, uint32_t &by)
{
    const uint32_t gx = gridDim.x, n = gridDim.x * gridDim.y;
    const uint32_t id = blockIdx.x + blockIdx.y * gx;
    const uint32_t x = id % 8u, s = id / 8u, per = n / 8u, rem = n % 8u;
    const uint32_t t = x * per + (x < rem ? x : rem) + s;
    bx = t % gx;
    by = t / gx;
}

__device__ inline float4 ld_rgba(const void *p, int fmt, size_t i)
{
    if (fmt == DOF_RGBA32F) return reinterpret_cast<const float4 *>(p)[i];
    const __half *h = reinterpret_cast<const __half *>(p) + 4 * i;
    return make_float4(__half2float(h[0]), __half2float(h[1]), __half2float(h[2]), __half2float(h[3]));
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

__device__ inline float4 bilinear4(const float4 *img, int w, int h, float x, float y)
{
    float x0f = floorf(x), y0f = floorf(y);
    float fx = x - x0f, fy = y - y0f;
    int x0 = (int)x0f, y0 = (int)y0f;
    int x1 = clampi(x0 + 1, 0, w - 1), y1 = clampi(y0 + 1, 0, h - 1);
    x0 = clampi(x0, 0, w - 1);
    y0 = clampi(y0, 0, h - 1);
    // 32-bit texel indices: a frame has at most 2^30 pixels
    const float4 *r0 = img + (uint32_t)(y0 * w), *r1 = img + (uint32_t)(y1 * w);
    float4 a = r0[x0], b = r0[x1];
    float4 c = r1[x0], d = r1[x1];
    float4 top, bot, o;
    top.x = a.x + (b.x - a.x) * fx; bot.x = c.x + (d.x - c.x) * fx; o.x = top.x + (bot.x - top.x) * fy;
    top.y = a.y + (b.y - a.y) * fx; bot.y = c.y + (d.y - c.y) * fx; o.y = top.y + (bot.y - top.y) * fy;
    top.z = a.z + (b.z - a.z) * fx; bot.z = c.z + (d.z - c.z) * fx; o.z = top.z + (bot.z - top.z) * fy;
    top.w = a.w + (b.w - a.w) * fx; bot.w = c.w + (d.w - c.w) * fx; o.w = top.w + (bot.w - top.w) * fy;
    return o;
}

// bilinear4 where the caller has shown 0 <= x < w - 1 and 0 <= y < h - 1 and
// w < 2^24: no clamp changes an index, floor is the integer conversion, and
// x - floor(x) is exact for x >= 0 (so fract gives the same bits), hence the
// same result with fewer instructions.
__device__ inline float4 bilinear4_in(const float4 *img, int w, float x, float y)
{
    const int x0 = (int)x, y0 = (int)y;
    const float fx = __builtin_amdgcn_fractf(x), fy = __builtin_amdgcn_fractf(y);
    const float4 *r0 = img + (uint32_t)(__umul24(y0, w) + x0), *r1 = r0 + w;
    float4 a = r0[0], b = r0[1];
    float4 c = r1[0], d = r1[1];
    float4 top, bot, o;
    top.x = a.x + (b.x - a.x) * fx; bot.x = c.x + (d.x - c.x) * fx; o.x = top.x + (bot.x - top.x) * fy;
    top.y = a.y + (b.y - a.y) * fx; bot.y = c.y + (d.y - c.y) * fx; o.y = top.y + (bot.y - top.y) * fy;
    top.z = a.z + (b.z - a.z) * fx; bot.z = c.z + (d.z - c.z) * fx; o.z = top.z + (bot.z - top.z) * fy;
    top.w = a.w + (b.w - a.w) * fx; bot.w = c.w + (d.w - c.w) * fx; o.w = top.w + (bot.w - top.w) * fy;
    return o;
}

__device__ inline int nearest_idx(float s, int n) { return clampi((int)floorf(s + 0.5f), 0, n - 1); }

// Median of 9 by a max-min exchange network (19 compare-exchanges).
__device__ inline float median9(float p0, float p1, float p2, float p3, float p4, float p5, float p6, float p7,
                                float p8)
{
#define DOF_CX(a, b)                  \
    {                                 \
        float lo_ = fmin_cs(a, b);    \
        float hi_ = fmax_cs(a, b);    \
        a = lo_;                      \
        b = hi_;                      \
    }
    DOF_CX(p1, p2); DOF_CX(p4, p5); DOF_CX(p7, p8);
    DOF_CX(p0, p1); DOF_CX(p3, p4); DOF_CX(p6, p7);
    DOF_CX(p1, p2); DOF_CX(p4, p5); DOF_CX(p7, p8);
    DOF_CX(p0, p3); DOF_CX(p5, p8); DOF_CX(p4, p7);
    DOF_CX(p3, p6); DOF_CX(p1, p4); DOF_CX(p2, p5);
    DOF_CX(p4, p7); DOF_CX(p4, p2); DOF_CX(p6, p4);
    DOF_CX(p4, p2);
#undef DOF_CX
    return p4;
}

// Half-res texel of the previous view that sees p (a direction when is_dir).
__device__ inline int reproject(const ViewConst &pv, int hw, int hh, const float p[3], bool is_dir)
{
    float e[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) e[a] = is_dir ? p[a] : p[a] - pv.pos[a];
    float ex = (e[0] * pv.right[0] + e[1] * pv.right[1]) + e[2] * pv.right[2];
    float ey = (e[0] * pv.up[0] + e[1] * pv.up[1]) + e[2] * pv.up[2];
    float ez = (e[0] * pv.fwd[0] + e[1] * pv.fwd[1]) + e[2] * pv.fwd[2];
    if (!(ez > 0.0f)) return -1;
    float pu = (ex / ez) / pv.tanx;
    float pvv = (ey / ez) / pv.tany;
    float px = ((pu + 1.0f) * 0.5f) * (float)hw - 0.5f;
    float py = ((1.0f - pvv) * 0.5f) * (float)hh - 0.5f;
    float sx = px + 0.5f, sy = py + 0.5f;
    if (!(sx >= 0.0f && sx < (float)hw && sy >= 0.0f && sy < (float)hh)) return -1;
    return (int)floorf(sy) * hw + (int)floorf(sx);
}

// History planes: A (near rgb, h) | B (far rgb, age) | C (cN, cF, mu1, mu2) | D var
struct Hist {
    const float4 *A, *B, *C;
    const float *D;
};
struct HistW {
    float4 *A, *B, *C;
    float *D;
};
__device__ inline Hist hist_view(const void *h, size_t np)
{
    const float4 *p = reinterpret_cast<const float4 *>(h);
    return Hist{p, p + np, p + 2 * np, reinterpret_cast<const float *>(p + 3 * np)};
}
__device__ inline HistW hist_wview(void *h, size_t np)
{
    float4 *p = reinterpret_cast<float4 *>(h);
    return HistW{p, p + np, p + 2 * np, reinterpret_cast<float *>(p + 3 * np)};
}

}  // namespace

Planes planes(const FrameConst &fc, const ScratchLayout &L, char *s)
{
    size_t np = (size_t)fc.hw * fc.hh;
    Planes p;
    p.colr = reinterpret_cast<float4 *>(s + L.colr);
    p.zn = reinterpret_cast<float4 *>(s + L.zn);
    p.zh = reinterpret_cast<float *>(s + L.zh);
    p.tile_max = reinterpret_cast<float *>(s + L.tile_max);
    p.tile_dil = reinterpret_cast<float *>(s + L.tile_dil);
    p.pre = reinterpret_cast<float4 *>(s + L.pre);
    p.gather = reinterpret_cast<float4 *>(s + L.gather);
    p.ppmed = reinterpret_cast<float4 *>(s + L.ppmed);
    p.prev_idx = reinterpret_cast<int32_t *>(s + L.prev_idx);
    p.chunk_cnt = reinterpret_cast<uint2 *>(s + L.chunk_cnt);
    p.chunk_off = reinterpret_cast<uint2 *>(s + L.chunk_off);
    p.counters = reinterpret_cast<uint32_t *>(s + L.counters);
    p.queue = reinterpret_cast<uint32_t *>(s + L.queue);
    p.ray_base = reinterpret_cast<uint32_t *>(s + L.ray_base);
    p.ray_pix = reinterpret_cast<uint32_t *>(s + L.ray_pix);
    const bool rec = fc.ray_records != 0;
    p.ray_hit = rec ? reinterpret_cast<int32_t *>(s + L.ray_hit) : nullptr;
    p.ray_t = rec ? reinterpret_cast<float *>(s + L.ray_t) : nullptr;
    p.ray_col = rec ? reinterpret_cast<float4 *>(s + L.ray_col) : nullptr;
    p.ray_pos = rec ? reinterpret_cast<float4 *>(s + L.ray_pos) : nullptr;
    const size_t nr = np * (size_t)fc.m;
    p.rec0 = reinterpret_cast<float4 *>(s + L.ray_rec);
    p.rec1 = reinterpret_cast<float2 *>(p.rec0 + nr);
    p.ray_lt = reinterpret_cast<uint2 *>(s + L.ray_lt);
    float4 *res = reinterpret_cast<float4 *>(s + L.resolve);
    p.R0 = res; p.R1 = res + np; p.R2 = res + 2 * np; p.R3 = res + 3 * np;
    float4 *tmp = reinterpret_cast<float4 *>(s + L.temporal);
    p.T0 = tmp; p.T1 = tmp + np;
    p.var_blur = reinterpret_cast<float *>(s + L.var_blur);
    p.rtmed = reinterpret_cast<float4 *>(s + L.rtmed);
    p.mips = reinterpret_cast<float4 *>(s + L.mips);
    p.tap = reinterpret_cast<float2 *>(s + L.tap);
    p.gtex = reinterpret_cast<float4 *>(s + L.gtex);
    p.mask_raw = reinterpret_cast<uint8_t *>(s + L.mask_raw);
    p.comp = (fc.taa & DOF_TAA_FINAL) ? reinterpret_cast<float4 *>(s + L.comp) : nullptr;
    p.rast = (fc.taa & DOF_TAA_RASTER) ? reinterpret_cast<float4 *>(s + L.rast) : nullptr;
    p.pptaa = (fc.taa & DOF_TAA_POST) ? reinterpret_cast<float4 *>(s + L.pptaa) : nullptr;
    p.ppout = (fc.taa & DOF_TAA_POST) ? p.pptaa : p.ppmed;
    p.recon = reinterpret_cast<float4 *>(s + L.recon);
    return p;
}

dof_gbuffer resolved_gbuffer(const FrameConst &fc, const Planes &P, const dof_gbuffer &gb)
{
    dof_gbuffer g = gb;
    if (fc.taa & DOF_TAA_RASTER) {
        g.colour = P.rast;
        g.colour_format = DOF_RGBA32F;
    }
    return g;
}

namespace {


// ---------------------------------------------------------------- A1

__device__ inline void b_reduce(const FrameConst &fc, const dof_gbuffer &gb, const Planes &P, const uint32_t bx, const uint32_t by)
{
    const int x = bx * kTile + threadIdx.x, y = by * kTile + threadIdx.y;
    float ar = 0.0f;
    if (x < fc.hw && y < fc.hh) {
        const size_t W = (size_t)fc.W;
        size_t t[4] = {(size_t)(2 * y) * W + 2 * x, (size_t)(2 * y) * W + 2 * x + 1,
                       (size_t)(2 * y + 1) * W + 2 * x, (size_t)(2 * y + 1) * W + 2 * x + 1};
        float zz[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) zz[k] = gb.depth[t[k]];
        int sel = 0;
        float z = zz[0];
        if (zz[1] < z) { z = zz[1]; sel = 1; }
        if (zz[2] < z) { z = zz[2]; sel = 2; }
        if (zz[3] < z) { z = zz[3]; sel = 3; }
        float4 c0 = ld_rgba(gb.colour, gb.colour_format, t[0]), c1 = ld_rgba(gb.colour, gb.colour_format, t[1]);
        float4 c2 = ld_rgba(gb.colour, gb.colour_format, t[2]), c3 = ld_rgba(gb.colour, gb.colour_format, t[3]);
        size_t ts = sel == 0 ? t[0] : (sel == 1 ? t[1] : (sel == 2 ? t[2] : t[3]));
        float4 nn = ld_rgba(gb.normal, gb.normal_format, ts);
        float r = coc_px(fc.cock, fc.d, z) * 0.25f;
        r = fmin_cs(r, fc.r_max);
        r = z < fc.d ? -r : r;
        size_t i = (size_t)y * fc.hw + x;
        P.colr[i] = make_float4(((c0.x + c1.x) + (c2.x + c3.x)) * 0.25f, ((c0.y + c1.y) + (c2.y + c3.y)) * 0.25f,
                                ((c0.z + c1.z) + (c2.z + c3.z)) * 0.25f, r);
        P.zn[i] = make_float4(z, nn.x, nn.y, nn.z);
        P.zh[i] = z;
        ar = fabsf(r);
    }
    // per-tile maximum |r| (tile == block)
    __shared__ float red[4];
    const int tid = threadIdx.y * kTile + threadIdx.x;
    for (int o = 32; o >= 1; o >>= 1) ar = fmax_cs(ar, __shfl_xor(ar, o));
    if ((tid & 63) == 0) red[tid >> 6] = ar;
    __syncthreads();
    if (tid == 0) {
        float m = 0.0f;
        for (int k = 0; k < 4; ++k) m = fmax_cs(m, red[k]);
        P.tile_max[(size_t)by * fc.tw + bx] = m;
    }
}

__global__ __launch_bounds__(256) void k_reduce(FrameConst fc, dof_gbuffer gb, Planes P)
{
    b_reduce(fc, gb, P, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void kb_reduce(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridTiles, blockIdx.x, bx, by)];
    b_reduce(J.fc, J.gb, J.P, bx, by);
}

// ---------------------------------------------------------------- A2

__device__ inline void b_dilate(const FrameConst &fc, const Planes &P, const uint32_t bx, const uint32_t by)
{
    const int tx = bx * blockDim.x + threadIdx.x, ty = by * blockDim.y + threadIdx.y;
    if (tx >= fc.tw || ty >= fc.th) return;
    float m = 0.0f;
    for (int j = ty - fc.D; j <= ty + fc.D; ++j)
        for (int i = tx - fc.D; i <= tx + fc.D; ++i)
            if (i >= 0 && j >= 0 && i < fc.tw && j < fc.th) m = fmax_cs(m, P.tile_max[(size_t)j * fc.tw + i]);
    P.tile_dil[(size_t)ty * fc.tw + tx] = m;
}

__global__ void k_dilate(FrameConst fc, Planes P)
{
    b_dilate(fc, P, blockIdx.x, blockIdx.y);
}

__global__ void kb_dilate(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridDilate, blockIdx.x, bx, by)];
    b_dilate(J.fc, J.P, bx, by);
}

// ---------------------------------------------------------------- A3

__device__ inline void b_prefilter(const FrameConst &fc, const Planes &P, const uint32_t bx, const uint32_t by)
{
    const int x = bx * kBX + threadIdx.x, y = by * kBY + threadIdx.y;
    if (x >= fc.hw || y >= fc.hh) return;
    const size_t i = (size_t)y * fc.hw + x;
    float Rn = P.tile_dil[(size_t)(y / fc.T) * fc.tw + x / fc.T];
    float dpre = Rn * 0.25f;
    if (dpre < kSqrt2) dpre = kSqrt2;
    float sp = dpre * 0.5f;
    float rc = P.colr[i].w;
    float ax = 0.0f, ay = 0.0f, az = 0.0f, sw = 0.0f;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            float sx = (float)x + (float)dx * sp, sy = (float)y + (float)dy * sp;
            float4 v = bilinear4(P.colr, fc.hw, fc.hh, sx, sy);
            float w = 1.0f / (1.0f + fabsf(v.w - rc));
            ax = ax + w * v.x;
            ay = ay + w * v.y;
            az = az + w * v.z;
            sw = sw + w;
        }
    const float4 pre = make_float4(ax / sw, ay / sw, az / sw, rc);
    P.pre[i] = pre;
    // the texel as the gather's taps read it, one 16-byte load: colour, the
    // radius's magnitude (the only part the gather uses) and, in its sign
    // bit, whether the pixel counts as a bright (specular) sample of the
    // bokeh share
    const bool bright = luma709(pre.x, pre.y, pre.z) > fc.l_spec;
    P.gtex[i] = make_float4(pre.x, pre.y, pre.z, __uint_as_float(__float_as_uint(fabsf(rc)) | (bright ? 0x80000000u : 0u)));
}

__global__ __launch_bounds__(kBX *kBY) void k_prefilter(FrameConst fc, Planes P)
{
    b_prefilter(fc, P, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBX *kBY) void kb_prefilter(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridHalf, blockIdx.x, bx, by)];
    b_prefilter(J.fc, J.P, bx, by);
}

// ---------------------------------------------------------------- A4

// One block of 256 threads per 16 x 16 tile of half-res pixels, the tile of
// the neighbourhood-maximum CoC, so the kernel radius R_n and with it every
// tap offset is the same for the whole block.  Each tap's texel column
// (per pixel column of the tile) and row (per pixel row) are computed once
// per block into LDS tables, with the same binary32 operations as the
// per-pixel definition, so the nearest-texel decisions are identical.  Each
// tap is one 16-byte load of the prefilter's gather texel (colour, radius
// magnitude, bright flag).  Optionally (launch knob gather_window) a tile
// whose taps stay within a win x win texel window first stages that window
// (texels and depths) in LDS and reads its taps there, in a kernel of its
// own; the other tiles read their taps from global memory (L1/L2) in a
// kernel that needs little LDS and so keeps many waves resident.  On the
// 1080p and 4K workloads the global reads are faster (the tiles that fit a
// window are the ones whose centres need the depth term, and the staging
// kernel holds fewer waves), so no staging is the default.
//
// Per tap, with D_fg = [|r_i| > dist] and D_bg = D_fg and [|r_c| > dist]:
// the two weights of eq. (1) add up to alpha when D_bg holds (foreground and
// background shares of one tap), to alpha (1 - w_bg) when only D_fg holds,
// and to 0 otherwise, so one weighted sum replaces the two and w_bg (with its
// division) is evaluated only where it matters.  Sums are reassociated
// relative to the per-pixel definition (tolerance parity); the weights'
// zero/non-zero pattern, and so the empty-kernel fallback, is unchanged.
// Whether a tile's taps fit a win x win texel window (win 0: no staging).
__device__ inline bool gather_fits(float Rn, int win) { return win > 0 && kTile + 2 * ((int)ceilf(Rn) + 1) <= win; }

// The taps of one ring (one distance): kBg when some lane of the wave has a
// centre radius at or below the ring's distance, so that its background taps
// need w_bg (a wave-uniform choice; the depth load and the division run only
// then).  sampleAlpha = 1 / max(|r|, 1/2)^2 with a hardware reciprocal
// (weights are normalised by their sum; tolerance parity).
template <bool kLds, bool kBg>
__device__ inline void gather_ring(const Planes &P, const float4 *s_tex, const float *s_z, const short *ixt,
                                   const short *iyt, int hw, int k0, int k1, float dist, bool centre_far, float zc,
                                   float range, float &v0, float &v1, float &v2, float &sw, float &ss)
{
#pragma unroll 4
    for (int k = k0; k < k1; ++k) {
        const int ix = ixt[k * kTile], iy = iyt[k * kTile];
        float4 ci;
        uint32_t j = 0;
        if constexpr (kLds) {
            j = (uint32_t)(iy + ix);
            ci = s_tex[j];
        } else {
            j = __umul24((uint32_t)iy, (uint32_t)hw) + (uint32_t)ix;
            ci = P.gtex[j];
        }
        const float ari = fabsf(ci.w);
        const float mr = fmax_cs(ari, 0.5f);
        const float alpha = __builtin_amdgcn_rcpf(mr * mr);
        float wb = alpha;
        if constexpr (kBg) {
            const float zi = kLds ? s_z[j] : P.zh[j];
            wb = centre_far ? alpha : alpha * (1.0f - sat((zi - zc) / range));
        }
        const float w = ari > dist ? wb : 0.0f;
        v0 = fmaf(w, ci.x, v0);
        v1 = fmaf(w, ci.y, v1);
        v2 = fmaf(w, ci.z, v2);
        sw = sw + w;
        ss = ss + ((__float_as_uint(ci.w) >> 31) ? w : 0.0f);
    }
}

// kWin > 0: the LDS variant for the tiles that fit a kWin window; kWin = 0:
// the global variant for the tiles that do not fit fc.gather_win.
template <int kWin>
__device__ inline void b_gather(const FrameConst &fc, const Rings &rings, const Planes &P, const uint32_t tx,
                                const uint32_t ty)
{
    constexpr bool kLds = kWin > 0;
    // per tap: the texel column of each pixel column of the tile and the
    // texel row (LDS variant: window row times window width) of each pixel row
    __shared__ short s_ix[kRingTaps * kTile], s_iy[kRingTaps * kTile];
    __shared__ float4 s_tex[kLds ? kWin * kWin : 1];
    __shared__ float s_z[kLds ? kWin * kWin : 1];
    const int tid = threadIdx.x;
    const int x0 = (int)tx * kTile, y0 = (int)ty * kTile;
    const float Rn = P.tile_dil[(size_t)ty * fc.tw + tx];
    if (gather_fits(Rn, kLds ? kWin : fc.gather_win) != kLds) return;   // the other variant takes this tile
    // every tap lies within ceil(R_n) + 1 texels of its pixel (ring offsets <= 1 kernel radius)
    const int C = (int)ceilf(Rn) + 1;
    const int wx0 = max(x0 - C, 0), wx1 = min(x0 + kTile - 1 + C, fc.hw - 1);
    const int wy0 = max(y0 - C, 0), wy1 = min(y0 + kTile - 1 + C, fc.hh - 1);
    const int ww = wx1 - wx0 + 1;
    for (int e = tid; e < kRingTaps * 2 * kTile; e += 256) {
        const int k = e / (2 * kTile), c = e % (2 * kTile);
        if (c < kTile) {
            const int ix = nearest_idx((float)(x0 + c) + rings.ox[k] * Rn, fc.hw);
            s_ix[k * kTile + c] = (short)(kLds ? clampi(ix, wx0, wx1) - wx0 : ix);
        } else {
            const int iy = nearest_idx((float)(y0 + c - kTile) + rings.oy[k] * Rn, fc.hh);
            s_iy[k * kTile + c - kTile] = (short)(kLds ? (clampi(iy, wy0, wy1) - wy0) * ww : iy);
        }
    }
    if constexpr (kLds) {
        // rows of the window, 64 texels wide at a time (kWin <= 64)
        static_assert(kWin <= 64, "one pass of 64 columns per window row");
        const int c = tid & 63;
        if (c < ww)
            for (int r = tid >> 6; r <= wy1 - wy0; r += 4) {
                const size_t j = (size_t)(wy0 + r) * fc.hw + (wx0 + c);
                s_tex[r * ww + c] = P.gtex[j];
                s_z[r * ww + c] = P.zh[j];
            }
    }
    __syncthreads();
    const int lx = tid & (kTile - 1), ly = tid / kTile;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= fc.hw || y >= fc.hh) return;
    const size_t i = (size_t)y * fc.hw + x;
    const float4 c0 = P.pre[i];
    const float zc = P.zh[i], arc = fabsf(c0.w);
    float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f, sw = 0.0f, ss = 0.0f;
    // rings of 1, 8, 16, 24, 32 taps, each at one distance
    constexpr int kRingStart[6] = {0, 1, 9, 25, 49, 81};
#pragma unroll
    for (int ring = 0; ring < 5; ++ring) {
        const int k0 = kRingStart[ring], k1 = kRingStart[ring + 1];
        const float dist = Rn * rings.frac[k0];
        const bool centre_far = arc > dist;   // background taps need the centre's radius too
        if (__all(centre_far))
            gather_ring<kLds, false>(P, s_tex, s_z, s_ix + lx, s_iy + ly, fc.hw, k0, k1, dist, true, zc,
                                     fc.depth_range, v0, v1, v2, sw, ss);
        else
            gather_ring<kLds, true>(P, s_tex, s_z, s_ix + lx, s_iy + ly, fc.hw, k0, k1, dist, centre_far, zc,
                                    fc.depth_range, v0, v1, v2, sw, ss);
    }
    float4 o;
    if (sw > 0.0f) o = make_float4(v0 / sw, v1 / sw, v2 / sw, ss / sw);
    else o = make_float4(c0.x, c0.y, c0.z, 0.0f);
    P.gather[i] = o;
}

template <int kWin>
__global__ __launch_bounds__(256) void k_gather(FrameConst fc, Rings rings, Planes P)
{
    // every tile costs about the same, so contiguous bands per XCD stay
    // balanced and neighbouring tiles share their halo in one L2
    uint32_t bx, by;
    xcd_tile(bx, by);
    b_gather<kWin>(fc, rings, P, bx, by);
}

template <int kWin>
__global__ __launch_bounds__(256) void kb_gather(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridTiles, blockIdx.x, bx, by)];
    b_gather<kWin>(J.fc, J.grings, J.P, bx, by);
}

// Both variants of the gather: the LDS one for tiles that fit the window,
// the global one for the rest (grid: the tiles, or the batch's tile blocks).
template <class Launch>
void launch_gather_pair(int win, Launch launch)
{
    switch (win) {
    case 32: launch(std::integral_constant<int, 32>{}); break;
    case 40: launch(std::integral_constant<int, 40>{}); break;
    case 48: launch(std::integral_constant<int, 48>{}); break;
    default: break;
    }
    launch(std::integral_constant<int, 0>{});
}

// ---------------------------------------------------------------- A5

__device__ inline void b_median_pp(const FrameConst &fc, const Planes &P, const uint32_t bx, const uint32_t by)
{
    const int x = bx * kBX + threadIdx.x, y = by * kBY + threadIdx.y;
    if (x >= fc.hw || y >= fc.hh) return;
    float4 v[9];
    int n = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx)
            v[n++] = P.gather[(size_t)clampi(y + dy, 0, fc.hh - 1) * fc.hw + clampi(x + dx, 0, fc.hw - 1)];
    const size_t i = (size_t)y * fc.hw + x;
    P.ppmed[i] = make_float4(median9(v[0].x, v[1].x, v[2].x, v[3].x, v[4].x, v[5].x, v[6].x, v[7].x, v[8].x),
                             median9(v[0].y, v[1].y, v[2].y, v[3].y, v[4].y, v[5].y, v[6].y, v[7].y, v[8].y),
                             median9(v[0].z, v[1].z, v[2].z, v[3].z, v[4].z, v[5].z, v[6].z, v[7].z, v[8].z),
                             v[4].w);
}

__global__ __launch_bounds__(kBX *kBY) void k_median_pp(FrameConst fc, Planes P)
{
    b_median_pp(fc, P, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBX *kBY) void kb_median_pp(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridHalf, blockIdx.x, bx, by)];
    b_median_pp(J.fc, J.P, bx, by);
}

// ---------------------------------------------------------------- A6

constexpr int kMaskHalo = 4, kMaskL = kTile + 2 * kMaskHalo;   // 24 x 24 LDS cells

__device__ inline void b_mask(const FrameConst &fc, const Planes &P, const void *hist_in, uint8_t *mask, const uint32_t bx, const uint32_t by)
{
    __shared__ float4 F[kMaskL][kMaskL];
    __shared__ float4 Hh[kMaskL][kMaskL];
    __shared__ float4 B[kMaskL][kMaskL];
    const int hw = fc.hw, hh = fc.hh;
    const int ox = bx * kTile - kMaskHalo, oy = by * kTile - kMaskHalo;
    const int tid = threadIdx.y * kTile + threadIdx.x;
    // Cells hold values at clamped coordinates; a coordinate g maps to cell g - origin.
    for (int c = tid; c < kMaskL * kMaskL; c += 256) {
        int lx = c % kMaskL, ly = c / kMaskL;
        int gx = clampi(ox + lx, 0, hw - 1), gy = clampi(oy + ly, 0, hh - 1);
        float4 v = P.zn[(size_t)gy * hw + gx];
        F[ly][lx] = make_float4(fc.d / v.x, v.y, v.z, v.w);
    }
    __syncthreads();
    const float g5[5] = {0.0625f, 0.25f, 0.375f, 0.25f, 0.0625f};
    for (int c = tid; c < kMaskL * kMaskL; c += 256) {
        int lx = c % kMaskL, ly = c / kMaskL;
        if (lx < 2 || lx >= kMaskL - 2) continue;
        int cx = clampi(ox + lx, 0, hw - 1);
        float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        for (int j = 0; j < 5; ++j) {
            float4 v = F[ly][clampi(cx + j - 2, 0, hw - 1) - ox];
            acc.x = acc.x + g5[j] * v.x;
            acc.y = acc.y + g5[j] * v.y;
            acc.z = acc.z + g5[j] * v.z;
            acc.w = acc.w + g5[j] * v.w;
        }
        Hh[ly][lx] = acc;
    }
    __syncthreads();
    for (int c = tid; c < kMaskL * kMaskL; c += 256) {
        int lx = c % kMaskL, ly = c / kMaskL;
        if (lx < 2 || lx >= kMaskL - 2 || ly < 2 || ly >= kMaskL - 2) continue;
        int cy = clampi(oy + ly, 0, hh - 1);
        float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        for (int i = 0; i < 5; ++i) {
            float4 v = Hh[clampi(cy + i - 2, 0, hh - 1) - oy][lx];
            acc.x = acc.x + g5[i] * v.x;
            acc.y = acc.y + g5[i] * v.y;
            acc.z = acc.z + g5[i] * v.z;
            acc.w = acc.w + g5[i] * v.w;
        }
        B[ly][lx] = acc;
    }
    __syncthreads();
    const int x = bx * kTile + threadIdx.x, y = by * kTile + threadIdx.y;
    if (x >= hw || y >= hh) return;
    const float sm[5] = {1.0f, 4.0f, 6.0f, 4.0f, 1.0f};
    const float dv[5] = {-1.0f, -2.0f, 0.0f, 2.0f, 1.0f};
    float gx[4], gy[4];
    {
        float axv[4] = {0.0f, 0.0f, 0.0f, 0.0f}, ayv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int r = 0; r < 5; ++r) {
            int ly = clampi(y + r - 2, 0, hh - 1) - oy;
            float hx[4] = {0.0f, 0.0f, 0.0f, 0.0f}, hs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int k = 0; k < 5; ++k) {
                float4 v = B[ly][clampi(x + k - 2, 0, hw - 1) - ox];
                float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    hx[c] = hx[c] + dv[k] * vv[c];
                    hs[c] = hs[c] + sm[k] * vv[c];
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                axv[c] = axv[c] + sm[r] * hx[c];
                ayv[c] = ayv[c] + dv[r] * hs[c];
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            gx[c] = axv[c] * 0.0078125f;
            gy[c] = ayv[c] * 0.0078125f;
        }
    }
    float dd = sqrtf(gx[0] * gx[0] + gy[0] * gy[0]);
    float an = 0.0f;
    for (int c = 1; c < 4; ++c) an = an + (gx[c] * gx[c] + gy[c] * gy[c]);
    float dn = sqrtf(an);
    float xx = (dd + dn) * fc.s;
    float xn = sat(1.0f - 1.0f / (xx + 1.0f));
    const size_t i = (size_t)y * hw + x;
    const float z = P.zh[i];
    int pi = -1;
    const size_t np = (size_t)hw * hh;
    if (fc.have_hist) {
        float fv[3], Pw[3];
        pixel_dir(fc.cur, x, y, hw, hh, fv);
        bool isdir = !(z < INFINITY);
#pragma unroll
        for (int a = 0; a < 3; ++a) Pw[a] = isdir ? fv[a] : fc.cur.pos[a] + z * fv[a];
        pi = reproject(fc.prev, hw, hh, Pw, isdir);
        if (pi >= 0 && !(hist_view(hist_in, np).B[pi].w > 0.0f)) pi = -1;
    }
    P.prev_idx[i] = pi;
    float var_prev = pi >= 0 ? hist_view(hist_in, np).D[pi] : 0.0f;
    float xf = sat(xn + var_prev * fc.var_mask_w) * (float)fc.m;
    int cnt = (int)floorf(xf + 0.5f);
    int near_oof = (z < fc.d) && (coc_px(fc.cock, fc.d, z) > kSqrt2);
    int n = cnt > near_oof ? cnt : near_oof;
    if (n > fc.m) n = fc.m;
    if (fc.mask_mode == DOF_MASK_FIXED) n = n > 0 ? fc.m : 0;
    if (fc.mask_mode == DOF_MASK_ALL) n = fc.m;
    mask[i] = (uint8_t)n;
}

__global__ __launch_bounds__(256) void k_mask(FrameConst fc, Planes P, const void *hist_in, uint8_t *mask)
{
    b_mask(fc, P, hist_in, mask, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void kb_mask(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridTiles, blockIdx.x, bx, by)];
    b_mask(J.fc, J.P, J.hist_in, J.fc.mask_mode == DOF_MASK_DILATE ? J.P.mask_raw : J.mask, bx, by);
}

// ---------------------------------------------------------------- A6, dilated (5.3)
// One block per 16 x 16 tile: the tile's window of raw counts (radius R =
// its dilated max CoC radius, rounded up) goes to LDS, then a horizontal and
// a vertical running maximum give each pixel the largest count within R.

constexpr int kDilMax = 32;
constexpr int kDilSide = kTile + 2 * kDilMax;

__device__ inline void b_mask_dilate(const FrameConst &fc, const Planes &P, uint8_t *mask, const uint32_t bx,
                                     const uint32_t by)
{
    __shared__ uint8_t win[kDilSide * kDilSide];
    __shared__ uint8_t hor[kDilSide * kTile];
    const int hw = fc.hw, hh = fc.hh, tid = threadIdx.y * kTile + threadIdx.x;
    const int R = min((int)ceilf(P.tile_dil[(size_t)by * fc.tw + bx]), kDilMax);
    const int S = kTile + 2 * R;
    const int ox = (int)bx * kTile - R, oy = (int)by * kTile - R;
    for (int c = tid; c < S * S; c += kTile * kTile) {
        const int gx = ox + c % S, gy = oy + c / S;
        win[c] = (gx >= 0 && gy >= 0 && gx < hw && gy < hh) ? P.mask_raw[(size_t)gy * hw + gx] : (uint8_t)0;
    }
    __syncthreads();
    for (int c = tid; c < S * kTile; c += kTile * kTile) {
        const int row = c / kTile, col = c % kTile;
        uint8_t m = 0;
        for (int k = 0; k <= 2 * R; ++k) m = max(m, win[row * S + col + k]);
        hor[row * kTile + col] = m;
    }
    __syncthreads();
    const int x = (int)bx * kTile + threadIdx.x, y = (int)by * kTile + threadIdx.y;
    if (x >= hw || y >= hh) return;
    uint8_t m = 0;
    for (int k = 0; k <= 2 * R; ++k) m = max(m, hor[(threadIdx.y + k) * kTile + threadIdx.x]);
    mask[(size_t)y * hw + x] = m;
}

__global__ __launch_bounds__(256) void k_mask_dilate(FrameConst fc, Planes P, uint8_t *mask)
{
    b_mask_dilate(fc, P, mask, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void kb_mask_dilate(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridTiles, blockIdx.x, bx, by)];
    b_mask_dilate(J.fc, J.P, J.mask, bx, by);
}

// ---------------------------------------------------------------- A7

constexpr int kPixLds = 4096;   // staged ray->pixel entries per 256-pixel round (16 rays per pixel)
// Chunks of 1024 pixels in row-major order; ranks from wave ballots (masked
// pixels) and wave prefix sums (rays), so the queue is ascending.

__device__ inline uint32_t wave_incl_scan(uint32_t v, int lane)
{
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    return v;
}

__device__ inline void b_compact_count(int64_t np, const uint8_t *__restrict__ mask, const Planes &P, const uint32_t bx, const uint32_t by)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    size_t base = (size_t)bx * kChunk;
    uint32_t cp = 0, cr = 0;
    for (int r = 0; r < kChunk / 256; ++r) {
        size_t i = base + (size_t)r * 256 + tid;
        uint32_t n = i < (size_t)np ? mask[i] : 0u;
        cp += n > 0u;
        cr += n;
    }
    for (int o = 32; o >= 1; o >>= 1) {
        cp += __shfl_xor(cp, o);
        cr += __shfl_xor(cr, o);
    }
    __shared__ uint32_t sp[4], sr[4];
    if (lane == 0) { sp[w] = cp; sr[w] = cr; }
    __syncthreads();
    if (tid == 0) P.chunk_cnt[bx] = make_uint2(sp[0] + sp[1] + sp[2] + sp[3], sr[0] + sr[1] + sr[2] + sr[3]);
}

__global__ __launch_bounds__(256) void k_compact_count(int64_t np, const uint8_t *__restrict__ mask, Planes P)
{
    // the traversal's counters start the frame at zero (the totals of the
    // compaction are written by its last scatter block)
    if (blockIdx.x == 0 && threadIdx.x < kWorkParts) {
        uint32_t *w = P.counters + kCntWork + threadIdx.x * kWorkStride;
        w[0] = 0u;
        for (int k = 0; k < kStatWords; ++k) w[kStatAt + k] = 0u;
    }
    b_compact_count(np, mask, P, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void kb_compact_count(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridChunk, blockIdx.x, bx, by)];
    b_compact_count((int64_t)J.fc.hw * J.fc.hh, J.mask, J.P, bx, by);
}

__device__ inline void b_compact_scan(int64_t nchunks, const Planes &P)
{
    __shared__ uint32_t pp[1024], pr[1024];
    const int per = (int)((nchunks + 1023) / 1024);
    const int b = threadIdx.x * per, e = (int)min((int64_t)(b + per), nchunks);
    uint32_t sp = 0, sr = 0;
    for (int i = b; i < e; ++i) {
        uint2 c = P.chunk_cnt[i];
        sp += c.x;
        sr += c.y;
    }
    pp[threadIdx.x] = sp;
    pr[threadIdx.x] = sr;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t a = threadIdx.x >= (unsigned)off ? pp[threadIdx.x - off] : 0u;
        uint32_t c = threadIdx.x >= (unsigned)off ? pr[threadIdx.x - off] : 0u;
        __syncthreads();
        pp[threadIdx.x] += a;
        pr[threadIdx.x] += c;
        __syncthreads();
    }
    uint32_t rp = pp[threadIdx.x] - sp, rr = pr[threadIdx.x] - sr;
    for (int i = b; i < e; ++i) {
        uint2 c = P.chunk_cnt[i];
        P.chunk_off[i] = make_uint2(rp, rr);
        rp += c.x;
        rr += c.y;
    }
    if (threadIdx.x == 1023) {
        P.counters[kCntMasked] = pp[1023];
        P.counters[kCntRays] = pr[1023];
    }
}

__global__ __launch_bounds__(1024) void kb_compact_scan(const Job *__restrict__ jobs)
{
    const Job &J = jobs[blockIdx.x];
    const int64_t np = (int64_t)J.fc.hw * J.fc.hh;
    b_compact_scan((np + kChunk - 1) / kChunk, J.P);
}

__device__ inline void b_compact_scatter(int64_t np, const uint8_t *__restrict__ mask, const Planes &P, const uint32_t bx,
                                         const uint32_t by, uint2 start)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    __shared__ uint32_t wp[4], wr[4];
    __shared__ uint32_t runp, runr;
    __shared__ uint32_t s_pix[kPixLds];   // ray -> queue position of one round's rays
    if (tid == 0) {
        runp = start.x;
        runr = start.y;
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    size_t base = (size_t)bx * kChunk;
    for (int r = 0; r < kChunk / 256; ++r) {
        size_t i = base + (size_t)r * 256 + tid;
        uint32_t n = i < (size_t)np ? mask[i] : 0u;
        uint64_t bal = __ballot(n > 0u);
        uint32_t rank = (uint32_t)__popcll(bal & lt);
        uint32_t incl = wave_incl_scan(n, lane);
        if (lane == 63) { wp[w] = (uint32_t)__popcll(bal); wr[w] = incl; }
        __syncthreads();
        uint32_t op = runp, orr = runr;
        const uint32_t rbase = runr, round_rays = wr[0] + wr[1] + wr[2] + wr[3];
        // the round's rays are one contiguous range: stage their pixel map in
        // LDS and store it coalesced (rounds with more rays store directly)
        const bool staged = round_rays <= (uint32_t)kPixLds;
        for (int k = 0; k < w; ++k) { op += wp[k]; orr += wr[k]; }
        if (n > 0u) {
            uint32_t pos = op + rank;
            uint32_t rb = orr + incl - n;
            P.queue[pos] = (uint32_t)i;
            P.ray_base[pos] = rb;
            if (staged) {
                for (uint32_t k = 0; k < n; ++k) s_pix[rb - rbase + k] = pos;
            } else {
                for (uint32_t k = 0; k < n; ++k) P.ray_pix[rb + k] = pos;
            }
        }
        __syncthreads();
        if (staged)
            for (uint32_t t = tid; t < round_rays; t += 256) P.ray_pix[rbase + t] = s_pix[t];
        if (tid == 0) {
            runp += wp[0] + wp[1] + wp[2] + wp[3];
            runr += wr[0] + wr[1] + wr[2] + wr[3];
        }
        __syncthreads();
    }
}

// A frame's scatter finds its chunk's offsets itself, summing the counts of
// the chunks before it (integer sums: the same offsets as a scan), so a
// frame needs no separate scan launch; the last chunk's block writes the
// totals.
__global__ __launch_bounds__(256) void k_compact_scatter(int64_t np, const uint8_t *__restrict__ mask, Planes P)
{
    __shared__ uint32_t sp[4], sr[4];
    const uint32_t bx = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t cp = 0, cr = 0;
    for (uint32_t i = (uint32_t)tid; i < bx; i += 256) {
        const uint2 c = P.chunk_cnt[i];
        cp += c.x;
        cr += c.y;
    }
    for (int o = 32; o >= 1; o >>= 1) {
        cp += __shfl_xor(cp, o);
        cr += __shfl_xor(cr, o);
    }
    if (lane == 0) { sp[w] = cp; sr[w] = cr; }
    __syncthreads();
    const uint2 start = make_uint2(sp[0] + sp[1] + sp[2] + sp[3], sr[0] + sr[1] + sr[2] + sr[3]);
    if (bx == gridDim.x - 1 && tid == 0) {
        const uint2 c = P.chunk_cnt[bx];
        P.counters[kCntMasked] = start.x + c.x;
        P.counters[kCntRays] = start.y + c.y;
    }
    b_compact_scatter(np, mask, P, bx, blockIdx.y, start);
}

__global__ __launch_bounds__(256) void kb_compact_scatter(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridChunk, blockIdx.x, bx, by)];
    b_compact_scatter((int64_t)J.fc.hw * J.fc.hh, J.mask, J.P, bx, by, J.P.chunk_off[bx]);
}

// ---------------------------------------------------------------- A11

// ---------------------------------------------------------------- A12

__device__ inline void b_temporal(const FrameConst &fc, const Planes &P, const uint8_t *__restrict__ mask,
                                                       const void *hist_in, void *hist_out, const uint32_t bx, const uint32_t by)
{
    const int x = bx * kBX + threadIdx.x, y = by * kBY + threadIdx.y;
    const int hw = fc.hw, hh = fc.hh;
    if (x >= hw || y >= hh) return;
    const size_t np = (size_t)hw * hh, i = (size_t)y * hw + x;
    HistW ho = hist_wview(hist_out, np);
    const int n = mask[i];
    const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (n == 0) {
        P.T0[i] = z4; P.T1[i] = z4;
        ho.A[i] = z4; ho.B[i] = z4; ho.C[i] = z4;
        return;
    }
    const float4 r0 = P.R0[i], r1 = P.R1[i], r2 = P.R2[i], r3 = P.R3[i];
    const float N = r0.w, hcur = r1.w, nf = (float)n - N;
    const int pn = P.prev_idx[i];
    const bool vn = pn >= 0;
    float fpos[3];
    bool fvalid = r3.w > 0.0f;
    if (fvalid) {
        fpos[0] = r3.x; fpos[1] = r3.y; fpos[2] = r3.z;
    } else {
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
        int cnt = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int xx = x + dx, yy = y + dy;
                if ((dx == 0 && dy == 0) || xx < 0 || yy < 0 || xx >= hw || yy >= hh) continue;
                size_t k = (size_t)yy * hw + xx;
                if (mask[k]) {
                    float4 q3 = P.R3[k];
                    if (q3.w > 0.0f) {
                        a0 = a0 + q3.x; a1 = a1 + q3.y; a2 = a2 + q3.z;
                        ++cnt;
                    }
                }
            }
        if (cnt > 0) {
            fpos[0] = a0 / (float)cnt; fpos[1] = a1 / (float)cnt; fpos[2] = a2 / (float)cnt;
            fvalid = true;
        }
    }
    Hist hi = hist_view(hist_in, np);
    int pf = -1;
    if (fc.have_hist && fvalid) {
        pf = reproject(fc.prev, hw, hh, fpos, false);
        if (pf >= 0 && !(hi.B[pf].w > 0.0f)) pf = -1;
    }
    const bool vf = pf >= 0;
    const float ah = fc.alpha_h;
    float4 hNa = vn ? hi.A[pn] : z4, hNb = vn ? hi.B[pn] : z4, hNc = vn ? hi.C[pn] : z4;
    float4 hFb = vf ? hi.B[pf] : z4, hFc = vf ? hi.C[pf] : z4;
    const float cur_n[3] = {r0.x, r0.y, r0.z}, cur_f[3] = {r1.x, r1.y, r1.z};
    const float hn_[3] = {hNa.x, hNa.y, hNa.z}, hf_[3] = {hFb.x, hFb.y, hFb.z};
    float accN[3], accF[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        accN[c] = N > 0.0f ? (vn ? lerp1(cur_n[c], hn_[c], ah) : cur_n[c]) : (vn ? hn_[c] : 0.0f);
        accF[c] = nf > 0.0f ? (vf ? lerp1(cur_f[c], hf_[c], ah) : cur_f[c]) : (vf ? hf_[c] : 0.0f);
    }
    float accCN = N > 0.0f ? (vn ? lerp1(r2.x, hNc.x, ah) : r2.x) : (vn ? hNc.x : 0.0f);
    float accCF = nf > 0.0f ? (vf ? lerp1(r2.y, hFc.y, ah) : r2.y) : (vf ? hFc.y : 0.0f);
    float accH = vn ? lerp1(hcur, hNa.w, ah) : hcur;
    float huse = fc.motion ? hcur : accH;
    float crt[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) crt[c] = lerp1(accF[c], accN[c], huse);
    float ct = lerp1(accCF, accCN, huse);
    float l = luma709(crt[0], crt[1], crt[2]);
    float mu1 = vn ? lerp1(l, hNc.z, ah) : l;
    float mu2 = vn ? lerp1(l * l, hNc.w, ah) : l * l;
    float v = mu2 - mu1 * mu1;
    v = v > 0.0f ? v : 0.0f;
    float age = vn ? hNb.w + 1.0f : 1.0f;
    P.T0[i] = make_float4(crt[0], crt[1], crt[2], 1.0f);
    P.T1[i] = make_float4(ct, huse, v, 0.0f);
    ho.A[i] = make_float4(accN[0], accN[1], accN[2], accH);
    ho.B[i] = make_float4(accF[0], accF[1], accF[2], age);
    ho.C[i] = make_float4(accCN, accCF, mu1, mu2);
}

__global__ __launch_bounds__(kBX *kBY) void k_temporal(FrameConst fc, Planes P, const uint8_t *__restrict__ mask,
                                                       const void *hist_in, void *hist_out)
{
    b_temporal(fc, P, mask, hist_in, hist_out, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBX *kBY) void kb_temporal(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridHalf, blockIdx.x, bx, by)];
    b_temporal(J.fc, J.P, J.mask, J.hist_in, J.hist_out, bx, by);
}

// ---------------------------------------------------------------- A12 blur + A13 median, mips
// One wave per 8 x 8 tile: variance blur (3x3 binomial), 3x3 median of the
// ray-traced colour (invalid neighbours replaced by the centre), level 0 of
// the validity-weighted mip chain, then levels 1..3 of the tile from LDS;
// also the 8-byte record (CoC or -inf, hit ratio) that the reconstruction
// reads for each of its taps.

__device__ inline void b_blur_median_mips(const FrameConst &fc, const Planes &P, void *hist_out, const uint32_t bx, const uint32_t by)
{
    const int tx = threadIdx.x & 7, ty = threadIdx.x >> 3;
    const int x = bx * 8 + tx, y = by * 8 + ty;
    const int hw = fc.hw, hh = fc.hh;
    const size_t np = (size_t)hw * hh;
    __shared__ float4 m0[8][8];
    __shared__ float4 m1[4][4];
    __shared__ float4 m2[2][2];
    if (x < hw && y < hh) {
        const size_t i = (size_t)y * hw + x;
        const float g3[3] = {0.25f, 0.5f, 0.25f};
        float acc = 0.0f;
        for (int r = 0; r < 3; ++r) {
            size_t row = (size_t)clampi(y + r - 1, 0, hh - 1) * hw;
            float hs = 0.0f;
            for (int k = 0; k < 3; ++k) hs = hs + g3[k] * P.T1[row + clampi(x + k - 1, 0, hw - 1)].z;
            acc = acc + g3[r] * hs;
        }
        P.var_blur[i] = acc;
        hist_wview(hist_out, np).D[i] = acc;
        float4 c = P.T0[i];
        const float4 t1 = P.T1[i];
        P.tap[i] = make_float2(c.w > 0.0f ? t1.x : -INFINITY, t1.y);
        float4 med = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (c.w > 0.0f) {
            float4 v[9];
            int n = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    float4 t = P.T0[(size_t)clampi(y + dy, 0, hh - 1) * hw + clampi(x + dx, 0, hw - 1)];
                    v[n++] = t.w > 0.0f ? t : c;
                }
            med = make_float4(median9(v[0].x, v[1].x, v[2].x, v[3].x, v[4].x, v[5].x, v[6].x, v[7].x, v[8].x),
                              median9(v[0].y, v[1].y, v[2].y, v[3].y, v[4].y, v[5].y, v[6].y, v[7].y, v[8].y),
                              median9(v[0].z, v[1].z, v[2].z, v[3].z, v[4].z, v[5].z, v[6].z, v[7].z, v[8].z),
                              1.0f);
        }
        P.rtmed[i] = med;
        float4 pm = make_float4(med.x * med.w, med.y * med.w, med.z * med.w, med.w);
        P.mips[fc.moff[0] + i] = pm;
        m0[ty][tx] = pm;
    }
    __syncthreads();
    // level 1 (4 x 4 of this tile)
    if (threadIdx.x < 16) {
        const int lx = threadIdx.x & 3, ly = threadIdx.x >> 2;
        const int gx = bx * 4 + lx, gy = by * 4 + ly;
        if (gx < fc.mw[1] && gy < fc.mh[1]) {
            int x0 = 2 * gx, y0 = 2 * gy, x1 = clampi(2 * gx + 1, 0, fc.mw[0] - 1), y1 = clampi(2 * gy + 1, 0, fc.mh[0] - 1);
            float4 a = m0[y0 - by * 8][x0 - bx * 8], b = m0[y0 - by * 8][x1 - bx * 8];
            float4 c = m0[y1 - by * 8][x0 - bx * 8], d = m0[y1 - by * 8][x1 - bx * 8];
            float4 o = make_float4(((a.x + b.x) + (c.x + d.x)) * 0.25f, ((a.y + b.y) + (c.y + d.y)) * 0.25f,
                                   ((a.z + b.z) + (c.z + d.z)) * 0.25f, ((a.w + b.w) + (c.w + d.w)) * 0.25f);
            P.mips[fc.moff[1] + (size_t)gy * fc.mw[1] + gx] = o;
            m1[ly][lx] = o;
        }
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int lx = threadIdx.x & 1, ly = threadIdx.x >> 1;
        const int gx = bx * 2 + lx, gy = by * 2 + ly;
        if (gx < fc.mw[2] && gy < fc.mh[2]) {
            int x0 = 2 * gx, y0 = 2 * gy, x1 = clampi(2 * gx + 1, 0, fc.mw[1] - 1), y1 = clampi(2 * gy + 1, 0, fc.mh[1] - 1);
            float4 a = m1[y0 - by * 4][x0 - bx * 4], b = m1[y0 - by * 4][x1 - bx * 4];
            float4 c = m1[y1 - by * 4][x0 - bx * 4], d = m1[y1 - by * 4][x1 - bx * 4];
            float4 o = make_float4(((a.x + b.x) + (c.x + d.x)) * 0.25f, ((a.y + b.y) + (c.y + d.y)) * 0.25f,
                                   ((a.z + b.z) + (c.z + d.z)) * 0.25f, ((a.w + b.w) + (c.w + d.w)) * 0.25f);
            P.mips[fc.moff[2] + (size_t)gy * fc.mw[2] + gx] = o;
            m2[ly][lx] = o;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int gx = bx, gy = by;
        if (gx < fc.mw[3] && gy < fc.mh[3]) {
            int x0 = 2 * gx, y0 = 2 * gy, x1 = clampi(2 * gx + 1, 0, fc.mw[2] - 1), y1 = clampi(2 * gy + 1, 0, fc.mh[2] - 1);
            float4 a = m2[y0 - by * 2][x0 - bx * 2], b = m2[y0 - by * 2][x1 - bx * 2];
            float4 c = m2[y1 - by * 2][x0 - bx * 2], d = m2[y1 - by * 2][x1 - bx * 2];
            float4 o = make_float4(((a.x + b.x) + (c.x + d.x)) * 0.25f, ((a.y + b.y) + (c.y + d.y)) * 0.25f,
                                   ((a.z + b.z) + (c.z + d.z)) * 0.25f, ((a.w + b.w) + (c.w + d.w)) * 0.25f);
            P.mips[fc.moff[3] + (size_t)gy * fc.mw[3] + gx] = o;
        }
    }
}

__global__ __launch_bounds__(64) void k_blur_median_mips(FrameConst fc, Planes P, void *hist_out)
{
    b_blur_median_mips(fc, P, hist_out, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(64) void kb_blur_median_mips(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridMip, blockIdx.x, bx, by)];
    b_blur_median_mips(J.fc, J.P, J.hist_out, bx, by);
}

// ---------------------------------------------------------------- A13

// Tap positions are c + o * R with |o| <= 1 (ring radii k/4, k <= 4), and
// rounding is monotone, so they lie in [c - R, c + R] as computed in binary32;
// every later coordinate map is monotone too, so testing the two ends bounds
// every tap.  taps_inside: the nearest-pixel lookup of the tap plane needs no
// clamp.  mip_taps_inside: the bilinear mip lookup at scale sc needs none and
// reads only non-negative coordinates.
__device__ inline bool taps_inside(int c, float R, int n)
{
    const float lo = (float)c + (-R), hi = (float)c + R;
    return lo + 0.5f >= 0.0f && hi + 0.5f < (float)n;
}

__device__ inline bool mip_taps_inside(int c, float R, float sc, int n)
{
    const float lo = (float)c + (-R), hi = (float)c + R;
    return (lo + 0.5f) * sc - 0.5f >= 0.0f && (hi + 0.5f) * sc - 0.5f < (float)(n - 1);
}

// Trilinear accumulation of one tap: the two mip levels' bilinear samples
// blended by the lod fraction, folded into eight texel weights (level 0
// scaled by f0 = 1 - fl, level 1 by f1 = fl, both 0 for a rejected tap) and
// summed with fused multiply-adds into the four channels.  Equal to the
// per-tap lerp of two bilinear lerps in exact arithmetic (the
// reconstruction's tolerance parity covers the rounding); which texels a tap
// reads, and whether it counts, are decided exactly as in the per-pixel
// definition.
struct Tex4 {
    float4 a, b, c, d;   // (x0, y0), (x1, y0), (x0, y1), (x1, y1)
};

__device__ inline void acc_bilinear(const Tex4 &t, float fx, float fy, float f, float &a0, float &a1, float &a2,
                                    float &a3)
{
    const float wy1 = fy * f, wy0 = f - wy1;
    const float wx0 = 1.0f - fx;
    const float w00 = wx0 * wy0, w10 = fx * wy0, w01 = wx0 * wy1, w11 = fx * wy1;
    a0 = fmaf(t.d.x, w11, fmaf(t.c.x, w01, fmaf(t.b.x, w10, fmaf(t.a.x, w00, a0))));
    a1 = fmaf(t.d.y, w11, fmaf(t.c.y, w01, fmaf(t.b.y, w10, fmaf(t.a.y, w00, a1))));
    a2 = fmaf(t.d.z, w11, fmaf(t.c.z, w01, fmaf(t.b.z, w10, fmaf(t.a.z, w00, a2))));
    a3 = fmaf(t.d.w, w11, fmaf(t.c.w, w01, fmaf(t.b.w, w10, fmaf(t.a.w, w00, a3))));
}

// The four texels of a bilinear lookup at (x, y) of a w x h level: clamped to
// the image, or (Inside) shown inside it by the caller.
template <bool Inside>
__device__ inline Tex4 fetch4(const float4 *img, int w, int h, float x, float y, float &fx, float &fy)
{
    Tex4 t;
    if (Inside) {
        const int x0 = (int)x, y0 = (int)y;
        fx = __builtin_amdgcn_fractf(x);
        fy = __builtin_amdgcn_fractf(y);
        const float4 *r0 = img + (__mul24(y0, w) + x0), *r1 = r0 + w;
        t.a = r0[0]; t.b = r0[1]; t.c = r1[0]; t.d = r1[1];
    } else {
        const float x0f = floorf(x), y0f = floorf(y);
        fx = x - x0f;
        fy = y - y0f;
        const int xi = (int)x0f, yi = (int)y0f;
        const int xa = clampi(xi, 0, w - 1), xb = clampi(xi + 1, 0, w - 1);
        const size_t ra = (size_t)clampi(yi, 0, h - 1) * w, rb = (size_t)clampi(yi + 1, 0, h - 1) * w;
        t.a = img[ra + xa]; t.b = img[ra + xb]; t.c = img[rb + xa]; t.d = img[rb + xb];
    }
    return t;
}

// The same from a level staged in LDS: t holds its rows b[2]..b[3] and
// columns b[0]..b[1], bw = b[1] - b[0] + 1 wide.  The box holds every index
// the block's taps reach after the clamp to the image (see b_recon), so
// clamping into the box gives the same texels as clamping into the image,
// and every LDS access stays inside the staged box.
template <bool Inside>
__device__ inline Tex4 fetch4_lds(const float4 *tex, const int *b, int bw, float x, float y, float &fx, float &fy)
{
    Tex4 t;
    if (Inside) {
        const int x0 = (int)x, y0 = (int)y;
        fx = __builtin_amdgcn_fractf(x);
        fy = __builtin_amdgcn_fractf(y);
        const float4 *r0 = tex + (__mul24(y0 - b[2], bw) + (x0 - b[0])), *r1 = r0 + bw;
        t.a = r0[0]; t.b = r0[1]; t.c = r1[0]; t.d = r1[1];
    } else {
        const float x0f = floorf(x), y0f = floorf(y);
        fx = x - x0f;
        fy = y - y0f;
        int x0 = (int)x0f, y0 = (int)y0f;
        const int x1 = clampi(x0 + 1, b[0], b[1]) - b[0], y1 = clampi(y0 + 1, b[2], b[3]) - b[2];
        x0 = clampi(x0, b[0], b[1]) - b[0];
        y0 = clampi(y0, b[2], b[3]) - b[2];
        const int r0 = y0 * bw, r1 = y1 * bw;
        t.a = tex[r0 + x0]; t.b = tex[r0 + x1]; t.c = tex[r1 + x0]; t.d = tex[r1 + x1];
    }
    return t;
}

// The 81 taps of one pixel in tap order, from global memory (Lds = false) or
// from the staged levels.  Every tap's fetches are issued (indices in
// bounds: clamped, or shown inside) and rejected taps weigh 0, so the loads
// of several taps can be in flight at once.
template <bool Inside, bool Lds>
__device__ inline void recon_taps(int x, int y, float Rr, float fl, float sc0, float sc1, int hw, int hh,
                                  const float4 *m0, int w0, int h0, const int *b0, const float4 *m1, int w1, int h1,
                                  const int *b1, const Rings &rings, const float2 *tap, float &a0, float &a1,
                                  float &a2, float &a3, float &sh, int &na)
{
    const float omf = 1.0f - fl;
#pragma unroll 3
    for (int k = 0; k < kRingTaps; ++k) {
        float dist = Rr * rings.frac[k];
        float sx = (float)x + rings.ox[k] * Rr, sy = (float)y + rings.oy[k] * Rr;
        size_t j;
        if (Inside)
            j = (uint32_t)(__umul24((int)(sy + 0.5f), hw) + (int)(sx + 0.5f));
        else
            j = (size_t)nearest_idx(sy, hh) * hw + nearest_idx(sx, hw);
        // a tap counts when its pixel is ray traced and its CoC radius
        // reaches the tap (invalid pixels carry -inf)
        const float2 tj = tap[j];
        const bool ok = tj.x * 0.25f >= dist;
        const float u0 = (sx + 0.5f) * sc0 - 0.5f, v0 = (sy + 0.5f) * sc0 - 0.5f;
        const float u1 = (sx + 0.5f) * sc1 - 0.5f, v1 = (sy + 0.5f) * sc1 - 0.5f;
        float fx0, fy0, fx1, fy1;
        const Tex4 t0 = Lds ? fetch4_lds<Inside>(m0, b0, w0, u0, v0, fx0, fy0) : fetch4<Inside>(m0, w0, h0, u0, v0, fx0, fy0);
        const Tex4 t1 = Lds ? fetch4_lds<Inside>(m1, b1, w1, u1, v1, fx1, fy1) : fetch4<Inside>(m1, w1, h1, u1, v1, fx1, fy1);
        acc_bilinear(t0, fx0, fy0, ok ? omf : 0.0f, a0, a1, a2, a3);
        acc_bilinear(t1, fx1, fy1, ok ? fl : 0.0f, a0, a1, a2, a3);
        sh = sh + (ok ? tj.y : 0.0f);
        na += ok ? 1 : 0;
    }
}

constexpr int kReconLds = 2496;   // mip texels a block can stage in LDS (39 KB: 4 blocks per CU)

// Index range that the bilinear lookups of taps between coordinates lo and hi
// (one axis, already at the level's scale sc) reach after the clamp to
// [0, n - 1]: the coordinate map and floor are monotone, so the two ends bound
// every tap.
__device__ inline void mip_span(float lo, float hi, float sc, int n, int &a, int &b)
{
    a = clampi((int)floorf((lo + 0.5f) * sc - 0.5f), 0, n - 1);
    b = clampi((int)floorf((hi + 0.5f) * sc - 0.5f) + 1, 0, n - 1);
}

// Block of a frame's reconstruction: 16 x 16 pixels, whose square footprint
// stages fewer halo texels than a 64 x 4 row block (batches keep the common
// 64 x 4 pixel-kernel grid); the output does not depend on the shape.
constexpr int kReconBX = 16, kReconBY = 16;

template <int BX = kBX, int BY = kBY>
__device__ inline void b_recon(const FrameConst &fc, const Rings &rings, const Planes &P, const uint32_t bx, const uint32_t by)
{
    // The block's mip footprint: per level, the index box of every bilinear
    // lookup its pixels' taps make (taps lie within R of the pixel on both
    // axes), staged in LDS when the boxes fit; else the taps read the mips
    // in global memory.
    __shared__ float4 tex[kReconLds];
    __shared__ int box[4][4];   // per level: first and last column, first and last row
    __shared__ int base[5];     // per level: first LDS texel; [4]: texels in all
    const int tid = threadIdx.y * BX + threadIdx.x;
    if (tid < 4) {
        box[tid][0] = 0x7fffffff; box[tid][1] = -1;
        box[tid][2] = 0x7fffffff; box[tid][3] = -1;
    }
    __syncthreads();
    const int x = bx * BX + threadIdx.x, y = by * BY + threadIdx.y;
    const int hw = fc.hw, hh = fc.hh;
    const bool in = x < hw && y < hh;
    const size_t i = in ? (size_t)y * hw + x : 0;
    const bool traced = in && P.T0[i].w > 0.0f;
    float ct = 0.0f, hu = 0.0f, Rr = 0.0f, fl = 0.0f, sc0 = 1.0f, sc1 = 1.0f;
    int L0 = 0, L1 = 0;
    if (traced) {
        const float4 t1 = P.T1[i];
        ct = t1.x;
        hu = t1.y;
        Rr = fmin_cs(ct * 0.25f, fc.r_max);
        const float lod = clampf(ct * fc.lod_scale, 0.0f, fc.lod_max);
        L0 = (int)floorf(lod);
        const int Lmax = fc.lod_levels;
        if (L0 > Lmax) L0 = Lmax;
        L1 = L0 < Lmax ? L0 + 1 : Lmax;
        fl = lod - (float)L0;
        for (int L = 0; L < L0; ++L) sc0 = sc0 * 0.5f;
        for (int L = 0; L < L1; ++L) sc1 = sc1 * 0.5f;
        const float lx = (float)x + (-Rr), hx = (float)x + Rr, ly = (float)y + (-Rr), hy = (float)y + Rr;
        int c0, c1, r0, r1;
        mip_span(lx, hx, sc0, fc.mw[L0], c0, c1);
        mip_span(ly, hy, sc0, fc.mh[L0], r0, r1);
        atomicMin(&box[L0][0], c0); atomicMax(&box[L0][1], c1);
        atomicMin(&box[L0][2], r0); atomicMax(&box[L0][3], r1);
        mip_span(lx, hx, sc1, fc.mw[L1], c0, c1);
        mip_span(ly, hy, sc1, fc.mh[L1], r0, r1);
        atomicMin(&box[L1][0], c0); atomicMax(&box[L1][1], c1);
        atomicMin(&box[L1][2], r0); atomicMax(&box[L1][3], r1);
    }
    __syncthreads();
    if (tid == 0) {
        int n = 0;
        for (int L = 0; L < 4; ++L) {
            base[L] = n;
            if (box[L][1] >= box[L][0]) n += (box[L][1] - box[L][0] + 1) * (box[L][3] - box[L][2] + 1);
        }
        base[4] = n;
    }
    __syncthreads();
    const bool staged = base[4] <= kReconLds;
    if (staged) {
        for (int L = 0; L < 4; ++L) {
            if (box[L][1] < box[L][0]) continue;
            const int bw = box[L][1] - box[L][0] + 1, cnt = bw * (box[L][3] - box[L][2] + 1);
            const float4 *src = P.mips + fc.moff[L];
            for (int e = tid; e < cnt; e += BX * BY) {
                const int r = e / bw, c = e - r * bw;
                tex[base[L] + e] = src[(size_t)(box[L][2] + r) * fc.mw[L] + box[L][0] + c];
            }
        }
    }
    __syncthreads();
    if (!in) return;
    if (!traced) {
        P.recon[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, sh = 0.0f;
    int na = 0;
    const float4 *mip0 = P.mips + fc.moff[L0], *mip1 = P.mips + fc.moff[L1];
    const int w0 = fc.mw[L0], h0 = fc.mh[L0], w1 = fc.mw[L1], h1 = fc.mh[L1];
    // The interior paths are taken by a whole wave when every lane's taps
    // stay inside all planes it reads (same arithmetic, no clamps).
    const bool inside = hw < (1 << 24) && hh < (1 << 24) && taps_inside(x, Rr, hw) && taps_inside(y, Rr, hh) &&
                        mip_taps_inside(x, Rr, sc0, w0) && mip_taps_inside(y, Rr, sc0, h0) &&
                        mip_taps_inside(x, Rr, sc1, w1) && mip_taps_inside(y, Rr, sc1, h1);
    const bool all_inside = __ballot(!inside) == 0ull;
    if (staged) {
        const int bw0 = box[L0][1] - box[L0][0] + 1, bw1 = box[L1][1] - box[L1][0] + 1;
        if (all_inside)
            recon_taps<true, true>(x, y, Rr, fl, sc0, sc1, hw, hh, tex + base[L0], bw0, 0, box[L0], tex + base[L1], bw1,
                                   0, box[L1], rings, P.tap, a0, a1, a2, a3, sh, na);
        else
            recon_taps<false, true>(x, y, Rr, fl, sc0, sc1, hw, hh, tex + base[L0], bw0, 0, box[L0], tex + base[L1],
                                    bw1, 0, box[L1], rings, P.tap, a0, a1, a2, a3, sh, na);
    } else {
        if (all_inside)
            recon_taps<true, false>(x, y, Rr, fl, sc0, sc1, hw, hh, mip0, w0, h0, nullptr, mip1, w1, h1, nullptr, rings,
                                    P.tap, a0, a1, a2, a3, sh, na);
        else
            recon_taps<false, false>(x, y, Rr, fl, sc0, sc1, hw, hh, mip0, w0, h0, nullptr, mip1, w1, h1, nullptr, rings,
                                     P.tap, a0, a1, a2, a3, sh, na);
    }
    const float4 med = P.rtmed[i];
    float nb0 = a3 > 0.0f ? a0 / a3 : med.x, nb1 = a3 > 0.0f ? a1 / a3 : med.y, nb2 = a3 > 0.0f ? a2 / a3 : med.z;
    float hnb = na > 0 ? sh / (float)na : hu;
    float bb = clampf(P.var_blur[i] * fc.var_recon_w, 0.0f, fc.b_max);
    P.recon[i] = make_float4(lerp1(med.x, nb0, bb), lerp1(med.y, nb1, bb), lerp1(med.z, nb2, bb), lerp1(hu, hnb, bb));
}

__global__ __launch_bounds__(kReconBX *kReconBY) void k_recon(FrameConst fc, Rings rings, Planes P)
{
    b_recon<kReconBX, kReconBY>(fc, rings, P, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBX *kBY) void kb_recon(const Job *__restrict__ jobs, int njobs, Rings rings)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridHalf, blockIdx.x, bx, by)];
    b_recon(J.fc, rings, J.P, bx, by);
}

// ---------------------------------------------------------------- A14

__device__ inline void b_composite(const FrameConst &fc, const Planes &P, const dof_gbuffer &gb, const dof_frame_out &out, const uint32_t bx, const uint32_t by)
{
    const int x = bx * kBX + threadIdx.x, y = by * kBY + threadIdx.y;
    if (x >= fc.W || y >= fc.H) return;
    const int hw = fc.hw, hh = fc.hh;
    const size_t p = (size_t)y * fc.W + x;
    const float z = gb.depth[p];
    const float c = coc_px(fc.cock, fc.d, z);
    const float hx = (float)x * 0.5f - 0.25f, hy = (float)y * 0.5f - 0.25f;
    const float4 pp = bilinear4(P.ppout, hw, hh, hx, hy);
    const float x0f = floorf(hx), y0f = floorf(hy);
    const float fx = hx - x0f, fy = hy - y0f;
    const int x0 = (int)x0f, y0 = (int)y0f;
    const int xs[2] = {clampi(x0, 0, hw - 1), clampi(x0 + 1, 0, hw - 1)};
    const int ys[2] = {clampi(y0, 0, hh - 1), clampi(y0 + 1, 0, hh - 1)};
    const float wts[4] = {(1.0f - fx) * (1.0f - fy), fx * (1.0f - fy), (1.0f - fx) * fy, fx * fy};
    float sw = 0.0f, rc0 = 0.0f, rc1 = 0.0f, rc2 = 0.0f, rh = 0.0f, rct = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        size_t j = (size_t)ys[k >> 1] * hw + xs[k & 1];
        // validity (exactly 0 or 1) and CoC (0 where invalid) from the tap record
        const float2 tp = P.tap[j];
        const bool valid = tp.x != -INFINITY;
        float wv = valid ? wts[k] : 0.0f;
        float4 rj = P.recon[j];
        sw = sw + wv;
        rc0 = rc0 + wv * rj.x;
        rc1 = rc1 + wv * rj.y;
        rc2 = rc2 + wv * rj.z;
        rh = rh + wv * rj.w;
        rct = rct + wv * (valid ? tp.x : 0.0f);
    }
    const bool rtv = sw > 0.0f;
    if (rtv) {
        rc0 = rc0 / sw; rc1 = rc1 / sw; rc2 = rc2 / sw;
        rh = rh / sw;
        rct = rct / sw;
    }
    float4 o;
    if (c <= kSqrt2 && (!rtv || rct < kSqrt2)) {
        float4 g = ld_rgba(gb.colour, gb.colour_format, p);
        o = make_float4(g.x, g.y, g.z, 1.0f);
    } else if (!rtv) {
        o = make_float4(pp.x, pp.y, pp.z, 1.0f);
    } else if (z < fc.d) {
        o = make_float4(lerp1(rc0, pp.x, pp.w), lerp1(rc1, pp.y, pp.w), lerp1(rc2, pp.z, pp.w), 1.0f);
    } else {
        float t = sat(rh / fc.h_edge);
        float w = (t * t) * (3.0f - 2.0f * t);
        if (fc.composite_literal)   // the literal reading: a high hit ratio favours the post-process colour
            o = make_float4(lerp1(rc0, pp.x, w), lerp1(rc1, pp.y, w), lerp1(rc2, pp.z, w), 1.0f);
        else
            o = make_float4(lerp1(pp.x, rc0, w), lerp1(pp.y, rc1, w), lerp1(pp.z, rc2, w), 1.0f);
    }
    if (fc.taa & DOF_TAA_FINAL) P.comp[p] = o;
    else st_rgba(out.colour, out.colour_format, p, o);
}

__global__ __launch_bounds__(kBX *kBY) void k_composite(FrameConst fc, Planes P, dof_gbuffer gb, dof_frame_out out)
{
    // The frame's counters are final once the traversal has run: the first
    // thread writes the caller's stats record (masked px, rays, and the sums
    // of the traversal's statistics slots).
    if (out.stats && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.y == 0 && threadIdx.x == 0) {
        unsigned long long v = 0ull, t = 0ull;
        uint32_t drops = 0u;
        for (int p = 0; p < kWorkParts; ++p) {
            const uint32_t *w = P.counters + kCntWork + p * kWorkStride + kStatAt;
            v += *reinterpret_cast<const unsigned long long *>(w);
            t += *reinterpret_cast<const unsigned long long *>(w + 2);
            drops += w[4];
        }
        dof_stats *o = out.stats;
        o->masked_px = P.counters[kCntMasked];
        o->rays = P.counters[kCntRays];
        o->node_visits = v;
        o->tri_tests = t;
        o->stack_spills = drops;
    }
    b_composite(fc, P, gb, out, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBX *kBY) void kb_composite(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridFull, blockIdx.x, bx, by)];
    b_composite(J.fc, J.P, J.gb, J.out, bx, by);
}

// Per-job stats records of a batch: masked pixels and rays of the job; the
// traversal statistics of a batch are kept once, in its head (the first
// thread sums the traversal's statistics slots there).
__global__ void kb_stats(BatchHead *head, const Job *__restrict__ jobs, int njobs)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) {
        unsigned long long v = 0ull, t = 0ull;
        for (int p = 0; p < kWorkParts; ++p) {
            const uint32_t *w = head->work + p * kWorkStride + kStatAt;
            v += *reinterpret_cast<const unsigned long long *>(w);
            t += *reinterpret_cast<const unsigned long long *>(w + 2);
        }
        head->visits = v;
        head->tests = t;
    }
    if (j >= njobs || !jobs[j].out.stats) return;
    const uint32_t *c = jobs[j].P.counters;
    dof_stats *o = jobs[j].out.stats;
    o->masked_px = c[kCntMasked];
    o->rays = c[kCntRays];
    o->node_visits = 0;
    o->tri_tests = 0;
}

// ---------------------------------------------------------------- TAA
// Temporal anti-aliasing stages (3.4, after Karis 2014).  One resolve: the
// current image's colour at (x, y) of a w x h grid is blended with the
// history image of the same grid, fetched bilinearly where the pixel's point
// (view depth z through the jittered camera; its direction for the sky)
// lands in the previous camera -- none behind it or off the grid -- that
// history clamped per RGB channel to the current 3 x 3 range (clamp to
// edge), history weight 0.9.  cur(x, y) reads the current image.  The 4th
// channel is 1, or the current one's with keep_w.

__device__ inline size_t taa_plane_floats(const FrameConst &fc, int which)   // 0 final, 1 raster, 2 post-filter
{
    const size_t base = ((size_t)fc.hw * fc.hh * 13 + 3) & ~(size_t)3;   // the record, rounded up to 16 bytes
    return base + (size_t)which * 4 * (size_t)fc.W * fc.H;
}

template <class Cur>
__device__ inline float4 taa_resolve(const FrameConst &fc, const Cur &cur, float z, int x, int y, int w, int h,
                                     const float4 *hin, bool keep_w)
{
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const float4 v = cur(clampi(x + dx, 0, w - 1), clampi(y + dy, 0, h - 1));
            const float vv[3] = {v.x, v.y, v.z};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                mn[c] = vv[c] < mn[c] ? vv[c] : mn[c];
                mx[c] = vv[c] > mx[c] ? vv[c] : mx[c];
            }
        }
    const float4 c0 = cur(x, y);
    bool valid = false;
    float4 hc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (hin) {
        float fv[3], Pw[3], e[3];
        pixel_dir(fc.cur, x, y, w, h, fv);
        const bool isdir = !(z < INFINITY);
#pragma unroll
        for (int a = 0; a < 3; ++a) Pw[a] = isdir ? fv[a] : fc.cur.pos[a] + z * fv[a];
#pragma unroll
        for (int a = 0; a < 3; ++a) e[a] = isdir ? Pw[a] : Pw[a] - fc.prev.pos[a];
        const float ex = (e[0] * fc.prev.right[0] + e[1] * fc.prev.right[1]) + e[2] * fc.prev.right[2];
        const float ey = (e[0] * fc.prev.up[0] + e[1] * fc.prev.up[1]) + e[2] * fc.prev.up[2];
        const float ez = (e[0] * fc.prev.fwd[0] + e[1] * fc.prev.fwd[1]) + e[2] * fc.prev.fwd[2];
        if (ez > 0.0f) {
            const float pu = (ex / ez) / fc.prev.tanx, pv = (ey / ez) / fc.prev.tany;
            const float px = ((pu + 1.0f) * 0.5f) * (float)w - 0.5f;
            const float py = ((1.0f - pv) * 0.5f) * (float)h - 0.5f;
            if (px + 0.5f >= 0.0f && px + 0.5f < (float)w && py + 0.5f >= 0.0f && py + 0.5f < (float)h) {
                hc = bilinear4(hin, w, h, px, py);
                valid = true;
            }
        }
    }
    const float cv[3] = {c0.x, c0.y, c0.z}, hv[3] = {hc.x, hc.y, hc.z};
    float o[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float v = cv[c];
        if (valid) {
            float t = hv[c];
            t = t > mn[c] ? t : mn[c];
            t = t < mx[c] ? t : mx[c];
            v = lerp1(cv[c], t, 0.9f);
        }
        o[c] = v;
    }
    return make_float4(o[0], o[1], o[2], keep_w ? c0.w : 1.0f);
}

__device__ inline const float4 *taa_history(const FrameConst &fc, const void *hist_in, int which)
{
    return (fc.have_hist && hist_in) ? reinterpret_cast<const float4 *>(static_cast<const float *>(hist_in) +
                                                                        taa_plane_floats(fc, which))
                                     : nullptr;
}

// The raster image before filtering (DOF_TAA_RASTER): G-buffer colour in,
// the resolved plane out (every later stage reads it).
__device__ inline void b_taa_raster(const FrameConst &fc, const Planes &P, const dof_gbuffer &gb, const void *hist_in,
                                    void *hist_out, const uint32_t bx, const uint32_t by)
{
    const int x = bx * kBX + threadIdx.x, y = by * kBY + threadIdx.y;
    const int W = fc.W, H = fc.H;
    if (x >= W || y >= H) return;
    const size_t p = (size_t)y * W + x;
    auto cur = [&](int xx, int yy) { return ld_rgba(gb.colour, gb.colour_format, (size_t)yy * W + xx); };
    const float4 r = taa_resolve(fc, cur, gb.depth[p], x, y, W, H, taa_history(fc, hist_in, 1), false);
    P.rast[p] = r;
    reinterpret_cast<float4 *>(static_cast<float *>(hist_out) + taa_plane_floats(fc, 1))[p] = r;
}

// The half-res post-filter output (DOF_TAA_POST); the quad's nearest depth
// locates each pixel.
__device__ inline void b_taa_post(const FrameConst &fc, const Planes &P, const void *hist_in, void *hist_out,
                                  const uint32_t bx, const uint32_t by)
{
    const int x = bx * kBX + threadIdx.x, y = by * kBY + threadIdx.y;
    const int hw = fc.hw, hh = fc.hh;
    if (x >= hw || y >= hh) return;
    const size_t i = (size_t)y * hw + x;
    auto cur = [&](int xx, int yy) { return P.ppmed[(size_t)yy * hw + xx]; };
    const float4 r = taa_resolve(fc, cur, P.zn[i].x, x, y, hw, hh, taa_history(fc, hist_in, 2), true);
    P.pptaa[i] = r;
    reinterpret_cast<float4 *>(static_cast<float *>(hist_out) + taa_plane_floats(fc, 2))[i] = r;
}

// The output after the composite (DOF_TAA_FINAL).
__device__ inline void b_taa_final(const FrameConst &fc, const Planes &P, const dof_gbuffer &gb, const void *hist_in,
                                   void *hist_out, const dof_frame_out &out, const uint32_t bx, const uint32_t by)
{
    const int x = bx * kBX + threadIdx.x, y = by * kBY + threadIdx.y;
    const int W = fc.W, H = fc.H;
    if (x >= W || y >= H) return;
    const size_t p = (size_t)y * W + x;
    auto cur = [&](int xx, int yy) { return P.comp[(size_t)yy * W + xx]; };
    const float4 r = taa_resolve(fc, cur, gb.depth[p], x, y, W, H, taa_history(fc, hist_in, 0), false);
    st_rgba(out.colour, out.colour_format, p, r);
    reinterpret_cast<float4 *>(static_cast<float *>(hist_out) + taa_plane_floats(fc, 0))[p] = r;
}

__global__ __launch_bounds__(kBX *kBY) void k_taa_raster(FrameConst fc, Planes P, dof_gbuffer gb, const void *hist_in,
                                                         void *hist_out)
{
    b_taa_raster(fc, P, gb, hist_in, hist_out, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBX *kBY) void k_taa_post(FrameConst fc, Planes P, const void *hist_in, void *hist_out)
{
    b_taa_post(fc, P, hist_in, hist_out, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBX *kBY) void k_taa_final(FrameConst fc, Planes P, dof_gbuffer gb, const void *hist_in,
                                                        void *hist_out, dof_frame_out out)
{
    b_taa_final(fc, P, gb, hist_in, hist_out, out, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBX *kBY) void kb_taa_raster(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridFull, blockIdx.x, bx, by)];
    b_taa_raster(J.fc, J.P, J.gb_in, J.hist_in, J.hist_out, bx, by);
}

__global__ __launch_bounds__(kBX *kBY) void kb_taa_post(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridHalf, blockIdx.x, bx, by)];
    b_taa_post(J.fc, J.P, J.hist_in, J.hist_out, bx, by);
}

__global__ __launch_bounds__(kBX *kBY) void kb_taa_final(const Job *__restrict__ jobs, int njobs)
{
    uint32_t bx, by;
    const Job &J = jobs[job_of_block(jobs, njobs, kGridFull, blockIdx.x, bx, by)];
    b_taa_final(J.fc, J.P, J.gb, J.hist_in, J.hist_out, J.out, bx, by);
}

__global__ void k_fill_zero(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

inline dim3 grid2(int w, int h, int bx, int by) { return dim3((w + bx - 1) / bx, (h + by - 1) / by); }

}  // namespace

#define DOF_REC(k)                                          \
    do {                                                    \
        if (ev) {                                           \
            hipError_t e_ = hipEventRecord(ev[(k)], st);    \
            if (e_ != hipSuccess) return e_;                \
        }                                                   \
    } while (0)

hipError_t launch_frame_pre(const FrameConst &fc, const Rings &rings, const ScratchLayout &L, char *scratch,
                            const dof_gbuffer &gb, const void *hist_in, void *hist_out, uint8_t *mask, hipEvent_t *ev,
                            const SideStream *side, hipStream_t st)
{
    Planes P = planes(fc, L, scratch);
    const int64_t np = (int64_t)fc.hw * fc.hh;
    DOF_REC(0);
    if (fc.taa & DOF_TAA_RASTER)
        k_taa_raster<<<grid2(fc.W, fc.H, kBX, kBY), dim3(kBX, kBY), 0, st>>>(fc, P, gb, hist_in, hist_out);
    k_reduce<<<dim3(fc.tw, fc.th), dim3(kTile, kTile), 0, st>>>(fc, resolved_gbuffer(fc, P, gb), P);
    DOF_REC(1);
    // the dilated tile radii feed the prefilter and the gather, and the ray
    // mask only in its dilated mode: otherwise the dilation heads the side chain
    const bool dil_side = side && fc.mask_mode != DOF_MASK_DILATE;
    if (!dil_side) k_dilate<<<grid2(fc.tw, fc.th, 16, 16), dim3(16, 16), 0, st>>>(fc, P);
    DOF_REC(2);
    // The post-process chain reads only the reduce's and the dilation's planes
    // and only the composite reads its result: with a side stream it is forked
    // after the ray generation, so it shares the GPU with the traversal and not
    // with the mask, compaction and generation that lead up to it.
    auto chain = [&](hipStream_t pst) -> hipError_t {
        if (dil_side) k_dilate<<<grid2(fc.tw, fc.th, 16, 16), dim3(16, 16), 0, pst>>>(fc, P);
        k_prefilter<<<grid2(fc.hw, fc.hh, kBX, kBY), dim3(kBX, kBY), 0, pst>>>(fc, P);
        DOF_REC(3);
        launch_gather_pair(fc.gather_win, [&](auto w) {
            k_gather<decltype(w)::value><<<dim3(fc.tw, fc.th), 256, 0, pst>>>(fc, rings, P);
        });
        DOF_REC(4);
        k_median_pp<<<grid2(fc.hw, fc.hh, kBX, kBY), dim3(kBX, kBY), 0, pst>>>(fc, P);
        if (fc.taa & DOF_TAA_POST)
            k_taa_post<<<grid2(fc.hw, fc.hh, kBX, kBY), dim3(kBX, kBY), 0, pst>>>(fc, P, hist_in, hist_out);
        return hipSuccess;
    };
    if (!side) {
        const hipError_t ec = chain(st);
        if (ec != hipSuccess) return ec;
    }
    DOF_REC(5);
    if (fc.mask_mode == DOF_MASK_DILATE) {
        k_mask<<<dim3(fc.tw, fc.th), dim3(kTile, kTile), 0, st>>>(fc, P, hist_in, P.mask_raw);
        k_mask_dilate<<<dim3(fc.tw, fc.th), dim3(kTile, kTile), 0, st>>>(fc, P, mask);
    } else {
        k_mask<<<dim3(fc.tw, fc.th), dim3(kTile, kTile), 0, st>>>(fc, P, hist_in, mask);
    }
    DOF_REC(6);
    k_compact_count<<<(unsigned)L.nchunks, 256, 0, st>>>(np, mask, P);
    k_compact_scatter<<<(unsigned)L.nchunks, 256, 0, st>>>(np, mask, P);
    const hipError_t e = launch_raygen(fc, L, scratch, st);
    if (e != hipSuccess) return e;
    DOF_REC(7);
    if (side) {
        hipError_t e2 = hipEventRecord(side->fork, st);
        if (e2 == hipSuccess) e2 = hipStreamWaitEvent(side->stream, side->fork, 0);
        if (e2 != hipSuccess) return e2;
        e2 = chain(side->stream);
        if (e2 == hipSuccess) e2 = hipEventRecord(side->join, side->stream);
        if (e2 != hipSuccess) return e2;
    }
    return hipGetLastError();
}

hipError_t launch_frame_post(const SceneDev &sd, const FrameConst &fc, const Rings &rings, const ScratchLayout &L, char *scratch,
                             const dof_gbuffer &gb, const void *hist_in, void *hist_out, uint8_t *mask,
                             const dof_frame_out &out, hipEvent_t *ev, const SideStream *side, hipStream_t st)
{
    Planes P = planes(fc, L, scratch);
    DOF_REC(8);
    {
        const hipError_t e = launch_shade_resolve(sd, fc, L, scratch, mask, st);
        if (e != hipSuccess) return e;
    }
    DOF_REC(9);
    k_temporal<<<grid2(fc.hw, fc.hh, kBX, kBY), dim3(kBX, kBY), 0, st>>>(fc, P, mask, hist_in, hist_out);
    DOF_REC(10);
    k_blur_median_mips<<<grid2(fc.hw, fc.hh, 8, 8), 64, 0, st>>>(fc, P, hist_out);
    DOF_REC(11);
    k_recon<<<grid2(fc.hw, fc.hh, kReconBX, kReconBY), dim3(kReconBX, kReconBY), 0, st>>>(fc, rings, P);
    DOF_REC(12);
    if (side) {
        const hipError_t e = hipStreamWaitEvent(st, side->join, 0);   // the post-process chain is done
        if (e != hipSuccess) return e;
    }
    k_composite<<<grid2(fc.W, fc.H, kBX, kBY), dim3(kBX, kBY), 0, st>>>(fc, P, resolved_gbuffer(fc, P, gb), out);
    if (fc.taa & DOF_TAA_FINAL)
        k_taa_final<<<grid2(fc.W, fc.H, kBX, kBY), dim3(kBX, kBY), 0, st>>>(fc, P, gb, hist_in, hist_out, out);
    DOF_REC(13);
    return hipGetLastError();
}

hipError_t launch_history_reset(float *hist, int64_t nfloats, hipStream_t st)
{
    k_fill_zero<<<1024, 256, 0, st>>>(hist, nfloats);
    return hipGetLastError();
}

hipError_t launch_batch_chain(const Job *jobs, int njobs, const uint32_t *nblk, const Rings &rings, bool with_dilate,
                              int taa, int gather_win, hipStream_t st)
{
    if (with_dilate) kb_dilate<<<nblk[kGridDilate], dim3(16, 16), 0, st>>>(jobs, njobs);
    kb_prefilter<<<nblk[kGridHalf], dim3(kBX, kBY), 0, st>>>(jobs, njobs);
    launch_gather_pair(gather_win, [&](auto w) {
        kb_gather<decltype(w)::value><<<nblk[kGridTiles], 256, 0, st>>>(jobs, njobs);
    });
    kb_median_pp<<<nblk[kGridHalf], dim3(kBX, kBY), 0, st>>>(jobs, njobs);
    if (taa & DOF_TAA_POST) kb_taa_post<<<nblk[kGridHalf], dim3(kBX, kBY), 0, st>>>(jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_batch_pre(const BatchHead *, const Job *jobs, int njobs, const uint32_t *nblk, const Rings &rings,
                            bool dilate, int taa, int gather_win, const SideStream *side, hipStream_t st)
{
    if (taa & DOF_TAA_RASTER) kb_taa_raster<<<nblk[kGridFull], dim3(kBX, kBY), 0, st>>>(jobs, njobs);
    kb_reduce<<<nblk[kGridTiles], dim3(kTile, kTile), 0, st>>>(jobs, njobs);
    // as in a frame: the dilation heads the side chain unless the ray mask
    // reads the dilated radii
    if (!side || dilate) kb_dilate<<<nblk[kGridDilate], dim3(16, 16), 0, st>>>(jobs, njobs);
    if (!side) {
        const hipError_t e = launch_batch_chain(jobs, njobs, nblk, rings, false, taa, gather_win, st);
        if (e != hipSuccess) return e;
    }
    kb_mask<<<nblk[kGridTiles], dim3(kTile, kTile), 0, st>>>(jobs, njobs);
    if (dilate) kb_mask_dilate<<<nblk[kGridTiles], dim3(kTile, kTile), 0, st>>>(jobs, njobs);
    kb_compact_count<<<nblk[kGridChunk], 256, 0, st>>>(jobs, njobs);
    kb_compact_scan<<<njobs, 1024, 0, st>>>(jobs);
    kb_compact_scatter<<<nblk[kGridChunk], 256, 0, st>>>(jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_batch_post(BatchHead *head, const Job *jobs, int njobs, const uint32_t *nblk, const Rings &rings,
                             int taa, const SideStream *side, hipStream_t st)
{
    {
        const hipError_t e = launch_batch_shade_resolve(jobs, njobs, nblk, st);
        if (e != hipSuccess) return e;
    }
    kb_temporal<<<nblk[kGridHalf], dim3(kBX, kBY), 0, st>>>(jobs, njobs);
    kb_blur_median_mips<<<nblk[kGridMip], 64, 0, st>>>(jobs, njobs);
    kb_recon<<<nblk[kGridHalf], dim3(kBX, kBY), 0, st>>>(jobs, njobs, rings);
    if (side) {
        const hipError_t e = hipStreamWaitEvent(st, side->join, 0);   // the post-process chain is done
        if (e != hipSuccess) return e;
    }
    kb_composite<<<nblk[kGridFull], dim3(kBX, kBY), 0, st>>>(jobs, njobs);
    if (taa & DOF_TAA_FINAL) kb_taa_final<<<nblk[kGridFull], dim3(kBX, kBY), 0, st>>>(jobs, njobs);
    kb_stats<<<(njobs + 127) / 128, 128, 0, st>>>(head, jobs, njobs);
    return hipGetLastError();
}

}  // namespace dof
