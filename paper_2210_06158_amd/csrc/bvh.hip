// LBVH build on the device: the acceleration structure that replaces the
// DXR build the paper times inside its Ray Trace pass (section 5.2).
//
//   leaf references (a triangle, or four clipped pieces of a long thin one:
//   early split clipping, Ernst & Greiner 2007) with their boxes ->
//   centroid bounds -> 64-bit keys (a large-box flag in bit 63 over a
//   63-bit Morton code, 21 bits per axis, of cubic cells) -> stable LSD
//   radix sort of (key, reference) -> binary radix tree over the 96-bit keys
//   key << 32 | reference (Karras 2012) -> the references' triangles
//   written in leaf order -> bottom-up refit of the child boxes stored in
//   each node.
//
// All results are bit-reproducible: min/max are compare-selects and the
// sort is stable, so the tree depends only on the input triangles.
#include "dof_internal.h"

namespace dof {
namespace {

constexpr int kThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kThreads * kSortItems;   // keys per sort block

__device__ inline void tri_box3(const float *v, float lo[3], float hi[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
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

__device__ inline float wave_min(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fmin_cs(v, __shfl_xor(v, o));
    return v;
}

__device__ inline float wave_max(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fmax_cs(v, __shfl_xor(v, o));
    return v;
}

// Box of the piece of triangle v inside the slab s0 <= x_k <= s1: on axis k
// the slab; on each other axis the range of the vertices inside the slab and
// of the points where edges cross its planes.  A crossing point is computed
// in binary32 and widened by 2^-20 (|edge extent| + |x|), more than its
// rounding error; the range is then clipped to the triangle's box.  So the
// box holds every point of the piece, and the pieces' boxes together hold
// the triangle: a ray that meets the triangle enters one of them.
__device__ inline void piece_box(const float *v, int k, float s0, float s1, const float lo[3], const float hi[3],
                                 float *out)
{
    out[k] = s0;
    out[3 + k] = s1;
    for (int m = 0; m < 3; ++m) {
        if (m == k) continue;
        float pl = INFINITY, ph = -INFINITY;
        for (int i = 0; i < 3; ++i) {
            const float vk = v[3 * i + k];
            if (vk >= s0 && vk <= s1) {
                const float x = v[3 * i + m];
                pl = x < pl ? x : pl;
                ph = x > ph ? x : ph;
            }
        }
        for (int e = 0; e < 3; ++e) {
            const float *p = v + 3 * e, *q = v + 3 * (e == 2 ? 0 : e + 1);
            for (int c = 0; c < 2; ++c) {
                const float pc = c ? s1 : s0;
                if ((p[k] < pc && pc < q[k]) || (q[k] < pc && pc < p[k])) {
                    const float t = (pc - p[k]) / (q[k] - p[k]);
                    const float d = q[m] - p[m];
                    const float x = p[m] + d * t;
                    const float g = (fabsf(d) + fabsf(x)) * 9.5367431640625e-07f;   // 2^-20
                    const float xl = x - g, xh = x + g;
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

// One thread per triangle: its references' boxes and triangle index.  A
// triangle with one reference keeps its own box; one with 2, 4 or 8 is cut
// into that many equal slabs of its box along the longest axis (the first
// one on ties).
__global__ __launch_bounds__(kThreads) void k_ref_emit(const float *__restrict__ verts, int nt,
                                                       const uint32_t *__restrict__ ref_off, float *__restrict__ boxes,
                                                       uint32_t *__restrict__ ref_tri)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= nt) return;
    float v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = verts[9 * (size_t)i + k];
    float lo[3], hi[3];
    tri_box3(v, lo, hi);
    const uint32_t r0 = ref_off[i], nr = ref_off[i + 1] - r0;
    if (nr == 1) {
        float *o = boxes + 6 * (size_t)r0;
        o[0] = lo[0]; o[1] = lo[1]; o[2] = lo[2];
        o[3] = hi[0]; o[4] = hi[1]; o[5] = hi[2];
        ref_tri[r0] = (uint32_t)i;
        return;
    }
    const float ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    int k = 0;
    if (ext[1] > ext[k]) k = 1;
    if (ext[2] > ext[k]) k = 2;
    const int np = nr <= 2 ? 2 : (nr <= 4 ? 4 : 8);   // 2, 4 or 8 (the host never writes another count)
    const float q = ext[k] * (1.0f / (float)np);
    float sl[9];
    sl[0] = lo[k];
    sl[np] = hi[k];
    for (int j = 1; j < np; ++j) {
        const float x = lo[k] + q * (float)j;
        sl[j] = x < hi[k] ? x : hi[k];
    }
    for (int j = 0; j < np; ++j) {
        float o[6];
        piece_box(v, k, sl[j], sl[j + 1], lo, hi, o);
        float *dst = boxes + 6 * (size_t)(r0 + j);
#pragma unroll
        for (int a = 0; a < 6; ++a) dst[a] = o[a];
        ref_tri[r0 + j] = (uint32_t)i;
    }
}

// Per-block min/max of reference-box centroids (grid-stride).
__global__ __launch_bounds__(kThreads) void k_centroid_bounds(const float *__restrict__ boxes, int n,
                                                              float *__restrict__ partial)
{
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        const float *bl = boxes + 6 * (size_t)i, *bh = bl + 3;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float c = (bl[a] + bh[a]) * 0.5f;
            lo[a] = fmin_cs(lo[a], c);
            hi[a] = fmax_cs(hi[a], c);
        }
    }
    __shared__ float red[6][kThreads / 64];
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float m = wave_min(lo[a]), M = wave_max(hi[a]);
        if (lane == 0) { red[a][w] = m; red[3 + a][w] = M; }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        int a = threadIdx.x;
        float r = red[a][0];
        for (int k = 1; k < kThreads / 64; ++k) r = a < 3 ? fmin_cs(r, red[a][k]) : fmax_cs(r, red[a][k]);
        partial[6 * blockIdx.x + a] = r;
    }
}

// Reduce the partial bounds.  Final slot: lo[3], then one scale for all three
// axes, inv = 2^21 / (largest extent), so Morton cells are cubes, then the
// squared-diagonal threshold above which a triangle counts as large
// (a quarter of the centre bounds' diagonal, squared).
__global__ __launch_bounds__(256) void k_bounds_final(float *__restrict__ partial, int nblocks)
{
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nblocks; b += 256)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin_cs(lo[a], partial[6 * b + a]);
            hi[a] = fmax_cs(hi[a], partial[6 * b + 3 + a]);
        }
    __shared__ float red[6][4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int a = 0; a < 3; ++a) {
        float m = wave_min(lo[a]), M = wave_max(hi[a]);
        if (lane == 0) { red[a][w] = m; red[3 + a][w] = M; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float l[3], ext[3];
        for (int a = 0; a < 3; ++a) {
            float lv = red[a][0], hv = red[3 + a][0];
            for (int k = 1; k < 4; ++k) { lv = fmin_cs(lv, red[a][k]); hv = fmax_cs(hv, red[3 + a][k]); }
            l[a] = lv;
            ext[a] = hv - lv;
        }
        const float e = fmax_cs(fmax_cs(ext[0], ext[1]), ext[2]);
        const float s2 = (ext[0] * ext[0] + ext[1] * ext[1]) + ext[2] * ext[2];
        float *out = partial + 6 * (size_t)nblocks;
        out[0] = l[0];
        out[1] = l[1];
        out[2] = l[2];
        out[3] = e > 0.0f ? 2097152.0f / e : 0.0f;
        out[4] = s2 * 0.0625f;
        out[5] = 0.0f;
    }
}

__device__ inline uint64_t spread_bits21(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ __launch_bounds__(kThreads) void k_morton(const float *__restrict__ boxes, int n,
                                                     const float *__restrict__ fin, uint64_t *__restrict__ keys,
                                                     uint32_t *__restrict__ ids)
{
    int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    float bl[3], bh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bl[a] = boxes[6 * (size_t)i + a];
        bh[a] = boxes[6 * (size_t)i + 3 + a];
    }
    uint32_t q[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float c = (bl[a] + bh[a]) * 0.5f;
        float t = floorf((c - fin[a]) * fin[3]);
        int qi = (int)t;
        q[a] = (uint32_t)(qi > 2097151 ? 2097151 : qi);
    }
    const float dx = bh[0] - bl[0], dy = bh[1] - bl[1], dz = bh[2] - bl[2];
    const uint64_t large = ((dx * dx + dy * dy) + dz * dz) > fin[4] ? 1ull : 0ull;
    keys[i] = (large << 63) | (spread_bits21(q[0]) << 2) | (spread_bits21(q[1]) << 1) | spread_bits21(q[2]);
    ids[i] = (uint32_t)i;
}

// ---------------------------------------------------------------- radix sort
// Per 8-bit pass: digit histogram per tile (digit-major), per-digit scans
// across tiles (one block per digit), a scan of the 256 digit totals, then a
// stable scatter.  Ranks inside a tile come from 8 wave ballots per round
// (lanes sharing a digit), so equal digits keep their input order.

__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint64_t *__restrict__ keys, int n, int shift,
                                                         uint32_t *__restrict__ hist, int nblocks)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    size_t base = (size_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        size_t i = base + (size_t)r * kThreads + threadIdx.x;
        if (i < (size_t)n) atomicAdd(&cnt[(uint32_t)(keys[i] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Block d: exclusive scan of digit d's counts over all tiles (in place); the
// digit total goes to tot[d].
__global__ __launch_bounds__(256) void k_scan_digit(uint32_t *__restrict__ hist, int nblocks,
                                                    uint32_t *__restrict__ tot)
{
    __shared__ uint32_t part[256];
    uint32_t *row = hist + (size_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (int c0 = 0; c0 < nblocks; c0 += 256) {
        const int i = c0 + threadIdx.x;
        const uint32_t v = i < nblocks ? row[i] : 0u;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            uint32_t u = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
            __syncthreads();
            part[threadIdx.x] += u;
            __syncthreads();
        }
        if (i < nblocks) row[i] = carry + part[threadIdx.x] - v;
        carry += part[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Exclusive scan of the 256 digit totals in place.
__global__ __launch_bounds__(256) void k_scan_totals(uint32_t *__restrict__ tot)
{
    __shared__ uint32_t part[256];
    const uint32_t v = tot[threadIdx.x];
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t u = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += u;
        __syncthreads();
    }
    tot[threadIdx.x] = part[threadIdx.x] - v;
}

__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                            const uint32_t *__restrict__ vin,
                                                            uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                            int n, int shift, const uint32_t *__restrict__ offs,
                                                            const uint32_t *__restrict__ doff, int nblocks)
{
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[kThreads / 64][256];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    running[tid] = doff[tid] + offs[(size_t)tid * nblocks + blockIdx.x];
#pragma unroll
    for (int k = 0; k < kThreads / 64; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    size_t base = (size_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        size_t i = base + (size_t)r * kThreads + tid;
        bool valid = i < (size_t)n;
        uint64_t key = valid ? kin[i] : 0ull;
        uint32_t val = valid ? vin[i] : 0u;
        uint32_t dg = (uint32_t)(key >> shift) & 0xffu;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            uint64_t bb = __ballot((dg >> bit) & 1u);
            match &= ((dg >> bit) & 1u) ? bb : ~bb;
        }
        uint32_t rank = (uint32_t)__popcll(match & lt);
        if (valid && rank == 0) wcnt[w][dg] = (uint32_t)__popcll(match);
        __syncthreads();
        if (valid) {
            uint32_t pos = running[dg] + rank;
            for (int k = 0; k < w; ++k) pos += wcnt[k][dg];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int k = 0; k < kThreads / 64; ++k) {
            add += wcnt[k][tid];
            wcnt[k][tid] = 0;
        }
        running[tid] += add;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- hierarchy

__global__ __launch_bounds__(kThreads) void k_reorder(const float *__restrict__ verts, const float *__restrict__ alb,
                                                      const uint32_t *__restrict__ ids,
                                                      const uint32_t *__restrict__ ref_tri, int n,
                                                      float4 *__restrict__ tris, float4 *__restrict__ albedo)
{
    int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    uint32_t id = ref_tri[ids[i]];
    const float *v = verts + 9 * (size_t)id;
    tris[3 * (size_t)i + 0] = make_float4(v[0], v[1], v[2], __uint_as_float(id));
    tris[3 * (size_t)i + 1] = make_float4(v[3], v[4], v[5], 0.0f);
    tris[3 * (size_t)i + 2] = make_float4(v[6], v[7], v[8], 0.0f);
    const float *a = alb + 3 * (size_t)id;
    albedo[i] = make_float4(a[0], a[1], a[2], 0.0f);
}

// Length of the common prefix of the 96-bit keys (code << 32 | reference) of
// leaves i and j; -1 outside the array.
__device__ inline int delta96(const uint64_t *keys, const uint32_t *ids, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    uint64_t x = keys[i] ^ keys[j];
    if (x != 0ull) return __clzll(x);
    return 64 + __clz(ids[i] ^ ids[j]);
}

__global__ __launch_bounds__(kThreads) void k_karras(const uint64_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ ids, int n,
                                                     BvhNode *__restrict__ nodes, uint32_t *__restrict__ parent,
                                                     uint32_t *__restrict__ flags, uint32_t *__restrict__ exit_count)
{
    int i = blockIdx.x * kThreads + threadIdx.x;
    if (i == 0) *exit_count = 0u;
    if (i >= n - 1) return;
    int dn = delta96(keys, ids, n, i, i + 1), dp = delta96(keys, ids, n, i, i - 1);
    int d = dn > dp ? 1 : -1;
    int dmin = d > 0 ? dp : dn;
    int lmax = 2;
    while (delta96(keys, ids, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta96(keys, ids, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = delta96(keys, ids, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (delta96(keys, ids, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int gamma = i + s * d + (d < 0 ? -1 : 0);
    int lo = i < j ? i : j, hi = i < j ? j : i;
    uint32_t left = (lo == gamma) ? ((uint32_t)gamma | kLeaf) : (uint32_t)gamma;
    uint32_t right = (hi == gamma + 1) ? ((uint32_t)(gamma + 1) | kLeaf) : (uint32_t)(gamma + 1);
    nodes[i].d = make_uint4(left, right, (uint32_t)lo, (uint32_t)hi);   // children, leaf range
    parent[(left & kLeaf) ? (size_t)(n - 1) + (left & ~kLeaf) : left] = (uint32_t)i;
    parent[(right & kLeaf) ? (size_t)(n - 1) + (right & ~kLeaf) : right] = (uint32_t)i;
    flags[i] = 0u;
    if (i == 0) parent[0] = ~0u;
}

__device__ inline void store_child_box(BvhNode *nd, bool left, const float lo[3], const float hi[3])
{
    if (left) {
        nd->a = make_float4(lo[0], hi[0], lo[1], hi[1]);
        nd->c.x = lo[2];
        nd->c.y = hi[2];
    } else {
        nd->b = make_float4(lo[0], hi[0], lo[1], hi[1]);
        nd->c.z = lo[2];
        nd->c.w = hi[2];
    }
}

// Refit: one thread per leaf climbs towards the root; the second thread to
// reach a node merges both child boxes and continues (compare-selects, left
// first), so every box is exact whatever the schedule.  Shared data must not
// need device-wide ordering per node: on a multi-die GPU an agent-scope
// acquire / release writes back and invalidates the die's L2.  So:
//  k_refit_local: a block owns kRefitThreads consecutive leaves; an internal
//    node whose leaf range lies inside them (its index is an end of its range,
//    so it is one of the block's indices) is finished within the block with
//    LDS arrival counters and the children's boxes in LDS.  A thread whose
//    next node's range leaves the block appends (child, node, box) to a list.
//  k_refit_top: one workgroup climbs from every list entry through the nodes
//    that span blocks (the kernel boundary publishes the first kernel's
//    writes; inside one workgroup, workgroup-scope ordering suffices).
// A full list (it holds exits_cap entries) makes a thread climb on with
// device-wide counters instead, which composes with the second kernel: that
// kernel only starts once every such climb has ended.
constexpr int kRefitThreads = 1024;

__device__ inline void union_lr(const float4 a, const float4 b, const float4 c, float lo[3], float hi[3])
{
    // union(left, right) as compare-selects, left first
    lo[0] = b.x < a.x ? b.x : a.x;
    hi[0] = b.y > a.y ? b.y : a.y;
    lo[1] = b.z < a.z ? b.z : a.z;
    hi[1] = b.w > a.w ? b.w : a.w;
    lo[2] = c.z < c.x ? c.z : c.x;
    hi[2] = c.w > c.y ? c.w : c.y;
}

__global__ __launch_bounds__(kRefitThreads) void k_refit_local(const float *__restrict__ ref_box,
                                                               const uint32_t *__restrict__ ids, int n, BvhNode *nodes,
                                                               const uint32_t *__restrict__ parent, uint32_t *flags,
                                                               uint4 *exits, uint32_t exits_cap, uint32_t *exit_count)
{
    __shared__ uint32_t lcnt[kRefitThreads];
    __shared__ float lbox[kRefitThreads][12];   // per in-block node: left lo xyz, hi xyz, then right
    const int tid = threadIdx.x;
    const uint32_t b0 = blockIdx.x * kRefitThreads, b1 = b0 + kRefitThreads;
    lcnt[tid] = 0u;
    __syncthreads();
    const int i = (int)b0 + tid;
    if (i >= n) return;
    // the leaf's box: its reference's
    const float *rb = ref_box + 6 * (size_t)ids[i];
    float lo[3] = {rb[0], rb[1], rb[2]}, hi[3] = {rb[3], rb[4], rb[5]};
    uint32_t child = (uint32_t)i | kLeaf;
    uint32_t p = parent[(size_t)(n - 1) + i];
    while (p != ~0u) {
        BvhNode *nd = nodes + p;
        const uint4 dd = nd->d;
        if (!(dd.z >= b0 && dd.w < b1)) break;   // the node's range leaves the block
        const bool is_left = dd.x == child;
        store_child_box(nd, is_left, lo, hi);
        float *slot = lbox[p - b0] + (is_left ? 0 : 6);
        slot[0] = lo[0]; slot[1] = lo[1]; slot[2] = lo[2];
        slot[3] = hi[0]; slot[4] = hi[1]; slot[5] = hi[2];
        const uint32_t old = __hip_atomic_fetch_add(&lcnt[p - b0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == 0u) return;
        const float *L = lbox[p - b0], *R = lbox[p - b0] + 6;
        lo[0] = R[0] < L[0] ? R[0] : L[0];
        hi[0] = R[3] > L[3] ? R[3] : L[3];
        lo[1] = R[1] < L[1] ? R[1] : L[1];
        hi[1] = R[4] > L[4] ? R[4] : L[4];
        lo[2] = R[2] < L[2] ? R[2] : L[2];
        hi[2] = R[5] > L[5] ? R[5] : L[5];
        child = p;
        p = parent[p];
    }
    if (p == ~0u) return;   // the whole tree lies in this block
    const uint32_t e = __hip_atomic_fetch_add(exit_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (e < exits_cap) {
        exits[2 * (size_t)e] = make_uint4(child, p, __float_as_uint(lo[0]), __float_as_uint(lo[1]));
        exits[2 * (size_t)e + 1] = make_uint4(__float_as_uint(lo[2]), __float_as_uint(hi[0]), __float_as_uint(hi[1]),
                                              __float_as_uint(hi[2]));
        return;
    }
    while (p != ~0u) {   // list full: device-wide counters
        BvhNode *nd = nodes + p;
        store_child_box(nd, nd->d.x == child, lo, hi);
        if (__hip_atomic_fetch_add(flags + p, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;
        union_lr(nd->a, nd->b, nd->c, lo, hi);
        child = p;
        p = parent[p];
    }
}

__global__ __launch_bounds__(kRefitThreads) void k_refit_top(BvhNode *nodes, const uint32_t *__restrict__ parent,
                                                             uint32_t *flags, const uint4 *__restrict__ exits,
                                                             uint32_t exits_cap, const uint32_t *__restrict__ exit_count)
{
    const uint32_t m = min(*exit_count, exits_cap);
    for (uint32_t e = threadIdx.x; e < m; e += kRefitThreads) {
        const uint4 e0 = exits[2 * (size_t)e], e1 = exits[2 * (size_t)e + 1];
        uint32_t child = e0.x, p = e0.y;
        float lo[3] = {__uint_as_float(e0.z), __uint_as_float(e0.w), __uint_as_float(e1.x)};
        float hi[3] = {__uint_as_float(e1.y), __uint_as_float(e1.z), __uint_as_float(e1.w)};
        while (p != ~0u) {
            BvhNode *nd = nodes + p;
            store_child_box(nd, nd->d.x == child, lo, hi);
            if (__hip_atomic_fetch_add(flags + p, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == 0u) break;
            union_lr(nd->a, nd->b, nd->c, lo, hi);
            child = p;
            p = parent[p];
        }
    }
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// The traversal's binary16 copy of the nodes.  Each plane is converted with
// directed rounding, low planes down and high planes up, and a result in the
// subnormal range goes outward to 0 or to the smallest normal (2^-14), so the
// copy holds every box whatever the device's binary16 denormal mode; a plane
// beyond the binary16 range becomes an infinite one on its side.
__device__ inline uint32_t half_bits(__half h) { return (uint32_t)__half_as_ushort(h); }

__device__ inline uint32_t plane_down(float x)
{
    const float m = 6.103515625e-05f;   // 2^-14, the smallest normal binary16
    float v = __half2float(__float2half_rd(x));
    if (v > 0.0f && v < m) v = 0.0f;
    else if (v < 0.0f && v > -m) v = -m;
    return half_bits(__float2half_rn(v));   // v is a binary16 value: exact
}

__device__ inline uint32_t plane_up(float x)
{
    const float m = 6.103515625e-05f;
    float v = __half2float(__float2half_ru(x));
    if (v > 0.0f && v < m) v = m;
    else if (v < 0.0f && v > -m) v = 0.0f;
    return half_bits(__float2half_rn(v));
}

__device__ inline uint32_t axis16(float lo, float hi) { return plane_down(lo) | (plane_up(hi) << 16); }

__global__ __launch_bounds__(kThreads) void k_nodes16(const BvhNode *__restrict__ nodes, int n, BvhNode16 *out)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const BvhNode nd = nodes[i];
    BvhNode16 o;
    o.a = make_uint4(axis16(nd.a.x, nd.a.y), axis16(nd.a.z, nd.a.w), axis16(nd.c.x, nd.c.y), axis16(nd.b.x, nd.b.y));
    o.b = make_uint4(axis16(nd.b.z, nd.b.w), axis16(nd.c.z, nd.c.w), nd.d.x, nd.d.y);
    out[i] = o;
}

}  // namespace

hipError_t launch_build_bvh(SceneDev &s, hipStream_t st)
{
    const int nt = s.ntri, n = s.nleaf;
    const int nb = s.bound_blocks;
    k_ref_emit<<<ceil_div(nt, kThreads), kThreads, 0, st>>>(s.verts_in, nt, s.ref_off, s.ref_box, s.ref_tri);
    k_centroid_bounds<<<nb, kThreads, 0, st>>>(s.ref_box, n, s.bounds);
    k_bounds_final<<<1, 256, 0, st>>>(s.bounds, nb);
    const float *fin = s.bounds + 6 * (size_t)nb;
    k_morton<<<ceil_div(n, kThreads), kThreads, 0, st>>>(s.ref_box, n, fin, s.keys, s.ids);
    const int sb = s.sort_blocks;
    uint32_t *doff = s.hist + 256 * (size_t)sb;
    uint64_t *ka = s.keys, *kb = s.keys_tmp;
    uint32_t *va = s.ids, *vb = s.ids_tmp;
    for (int shift = 0; shift < 64; shift += 8) {
        k_radix_hist<<<sb, kThreads, 0, st>>>(ka, n, shift, s.hist, sb);
        k_scan_digit<<<256, 256, 0, st>>>(s.hist, sb, doff);
        k_scan_totals<<<1, 256, 0, st>>>(doff);
        k_radix_scatter<<<sb, kThreads, 0, st>>>(ka, va, kb, vb, n, shift, s.hist, doff, sb);
        uint64_t *t = ka; ka = kb; kb = t;
        uint32_t *u = va; va = vb; vb = u;
    }
    k_reorder<<<ceil_div(n, kThreads), kThreads, 0, st>>>(s.verts_in, s.albedo_in, s.ids, s.ref_tri, n, s.tris,
                                                          s.albedo);
    if (n >= 2) {
        // the refit's list of block exits lives in the sort's spare key buffer (free after the sort)
        uint4 *exits = reinterpret_cast<uint4 *>(s.keys_tmp);
        const uint32_t cap = (uint32_t)((sizeof(uint64_t) * (size_t)n) / (2 * sizeof(uint4)));
        uint32_t *exit_count = s.aux + 8;
        k_karras<<<ceil_div(n - 1, kThreads), kThreads, 0, st>>>(s.keys, s.ids, n, s.nodes, s.parent, s.flags,
                                                                   exit_count);
        k_refit_local<<<ceil_div(n, kRefitThreads), kRefitThreads, 0, st>>>(s.ref_box, s.ids, n, s.nodes, s.parent,
                                                                              s.flags, exits, cap, exit_count);
        k_refit_top<<<1, kRefitThreads, 0, st>>>(s.nodes, s.parent, s.flags, exits, cap, exit_count);
        k_nodes16<<<ceil_div(n - 1, kThreads), kThreads, 0, st>>>(s.nodes, n - 1, s.nodes16);
    }
    return hipGetLastError();
}

}  // namespace dof
