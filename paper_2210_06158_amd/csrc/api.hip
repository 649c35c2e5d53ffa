// C ABI of libdof (include/dof.h): argument checks, buffer layouts, the
// lens-derived constants of a frame and the launch sequence.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "dof_internal.h"

struct dof_scene {
    dof::SceneDev dev;
    dof::SceneShade shade;
    char *arena;
    size_t arena_bytes;
    bool built;
    bool events_ready;   // ev[] created (host-side timing objects)
    bool timed_frame;    // ev[] hold the last timed frame
    hipEvent_t ev[DOF_NUM_STAGES + 1];
    bool side_ready;     // side holds a stream and two events
    dof::SideStream side;   // the post-process chain's stream (untimed frames)
};

namespace {

thread_local char g_err[512] = "";

dof_status vfail(dof_status code, const char *fmt, va_list ap)
{
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    return code;
}

dof_status fail(dof_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vfail(code, fmt, ap);
    va_end(ap);
    return code;
}

#define DOF_HIP(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(DOF_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// A roctx range over the host side of an entry point (its argument checks
// and launches); rocprofv3 --marker-trace records it, otherwise it costs a
// call into an inert library.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct SceneLayout {
    size_t verts_in, albedo_in, ref_off, ref_box, ref_tri, tris, albedo, nodes, nodes16, parent, keys, keys_tmp, ids,
        ids_tmp;
    size_t flags, hist, bounds, aux, total;
    int sort_blocks, bound_blocks;
};

// nt triangles, n leaf references
SceneLayout scene_layout(int64_t nt, int64_t n)
{
    SceneLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const int64_t ni = n > 1 ? n - 1 : 1;
    L.sort_blocks = (int)((n + 4095) / 4096);
    L.bound_blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
    L.verts_in = take(sizeof(float) * 9 * nt);
    L.albedo_in = take(sizeof(float) * 3 * nt);
    L.ref_off = take(sizeof(uint32_t) * (nt + 1));
    L.ref_box = take(sizeof(float) * 6 * n);
    L.ref_tri = take(sizeof(uint32_t) * n);
    L.tris = take(sizeof(float4) * 3 * n);
    L.albedo = take(sizeof(float4) * n);
    L.nodes = take(sizeof(dof::BvhNode) * ni);
    L.nodes16 = take(sizeof(dof::BvhNode16) * ni);
    L.parent = take(sizeof(uint32_t) * (2 * n - 1));
    L.keys = take(sizeof(uint64_t) * n);
    L.keys_tmp = take(sizeof(uint64_t) * n);
    L.ids = take(sizeof(uint32_t) * n);
    L.ids_tmp = take(sizeof(uint32_t) * n);
    L.flags = take(sizeof(uint32_t) * ni);
    L.hist = take(sizeof(uint32_t) * 256 * ((size_t)L.sort_blocks + 1));
    L.bounds = take(sizeof(float) * (6 * (size_t)L.bound_blocks + 8));
    L.aux = take(dof::kWorkBytes);
    L.total = off;
    return L;
}

// Leaf references (early split clipping, Ernst & Greiner 2007): with
// desc->leaf_split = s > 0 a triangle whose box's three face areas sum to more
// than 8 times its area -- a long thin slanted triangle, which most rays
// entering its box miss -- becomes 2^s references, its pieces in equal slabs
// of the box along the longest axis (clipped on the device when the BVH is
// built).  Decided here in binary64, so the size query and the upload agree.
constexpr int kMaxLeafSplit = 3;
constexpr int kMaxRefsPerTri = 1 << kMaxLeafSplit;

uint32_t refs_of(const float *v, int split)
{
    float lo[3], hi[3];
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
    double e[3], u[3], w[3];
    for (int a = 0; a < 3; ++a) {
        e[a] = (double)hi[a] - (double)lo[a];
        u[a] = (double)v[3 + a] - (double)v[a];
        w[a] = (double)v[6 + a] - (double)v[a];
    }
    const double faces = (e[0] * e[1] + e[1] * e[2]) + e[2] * e[0];
    const double cx = u[1] * w[2] - u[2] * w[1];
    const double cy = u[2] * w[0] - u[0] * w[2];
    const double cz = u[0] * w[1] - u[1] * w[0];
    const double c2 = (cx * cx + cy * cy) + cz * cz;
    return (c2 > 0.0 && faces * faces > 16.0 * c2) ? 1u << split : 1u;
}

// Reference offsets of the triangles (off may be NULL: count only); -1 when
// the references would not fit 31-bit leaf indices.
int64_t leaf_refs(const dof_scene_desc *desc, uint32_t *off)
{
    uint64_t acc = 0;
    for (int32_t i = 0; i < desc->ntri; ++i) {
        if (off) off[i] = (uint32_t)acc;
        acc += desc->leaf_split ? refs_of(desc->verts + 9 * (size_t)i, desc->leaf_split) : 1u;
        if (acc > (uint64_t)INT32_MAX) return -1;
    }
    if (off) off[desc->ntri] = (uint32_t)acc;
    return (int64_t)acc;
}

dof::ScratchLayout frame_layout(int W, int H, int m, int taa, int ray_records)
{
    dof::ScratchLayout L{};
    const size_t np = (size_t)(W / 2) * (H / 2);
    const int T = dof::kTile;
    const size_t ntiles = (size_t)((W / 2 + T - 1) / T) * ((H / 2 + T - 1) / T);
    const size_t nr = np * (size_t)m;
    L.nchunks = (int64_t)((np + dof::kChunk - 1) / dof::kChunk);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + (bytes ? bytes : 1));
        return o;
    };
    L.colr = take(16 * np);
    L.zn = take(16 * np);
    L.zh = take(4 * np);
    L.tile_max = take(4 * ntiles);
    L.tile_dil = take(4 * ntiles);
    L.pre = take(16 * np);
    L.gather = take(16 * np);
    L.ppmed = take(16 * np);
    L.gtex = take(16 * np);
    L.prev_idx = take(4 * np);
    L.mask_raw = take(np);
    L.chunk_cnt = take(8 * (size_t)L.nchunks);
    L.chunk_off = take(8 * (size_t)L.nchunks);
    L.counters = take(dof::kCountersBytes);
    L.queue = take(4 * np);
    L.ray_base = take(4 * np);
    L.ray_pix = take(4 * nr);
    L.ray_rec = take(24 * nr);   // a float4 and a float2 plane of nr
    L.ray_lt = take(8 * nr);
    if (ray_records) {   // per-ray hit id, distance, colour and position, for inspection only
        L.ray_hit = take(4 * nr);
        L.ray_t = take(4 * nr);
        L.ray_col = take(16 * nr);
        L.ray_pos = take(16 * nr);
    }
    L.resolve = take(64 * np);
    L.temporal = take(32 * np);
    L.var_blur = take(4 * np);
    L.rtmed = take(16 * np);
    size_t mt = 0;
    int w = W / 2, h = H / 2;
    for (int l = 0; l < 4; ++l) {
        mt += (size_t)w * h;
        w = (w + 1) >> 1;
        h = (h + 1) >> 1;
    }
    L.mips = take(16 * mt);
    L.tap = take(8 * np);
    L.recon = take(16 * np);
    L.comp = (taa & DOF_TAA_FINAL) ? take(16 * (size_t)W * H) : 0;   // composite colour before the final TAA
    L.rast = (taa & DOF_TAA_RASTER) ? take(16 * (size_t)W * H) : 0;  // raster colour after its TAA
    L.pptaa = (taa & DOF_TAA_POST) ? take(16 * np) : 0;              // post-filter output after its TAA
    L.total = off;
    return L;
}

struct LensDerived {
    float a, tanx, tany, cock, znb, ramp, half_a;
};

// Thin-lens constants (sections 1.1, 3.3): sensor at the focused image
// distance v = f d / (d - f); CoC(z) = (a f / (d - f)) (W / w_s) |1 - d / z|
// in pixels; eq. (6)'s near bound z_nb with w_i = W.
LensDerived lens_derived(const dof_lens &l, int W, int H)
{
    LensDerived q;
    const float f = l.focal, d = l.focus, ws = l.sensor;
    q.a = f / l.fnum;
    q.tanx = (ws * (d - f)) / ((2.0f * f) * d);
    q.tany = q.tanx * ((float)H / (float)W);
    q.cock = ((q.a * f) / (d - f)) * ((float)W / ws);
    const float g = (dof::kSqrt2 * (d - f)) * (ws / (float)W);
    const float af = q.a * f;
    q.znb = (af * d) / (af + g);
    q.ramp = 2.0f * (d - q.znb);
    q.half_a = q.a * 0.5f;
    return q;
}

// jitter: apply the camera's sub-pixel jitter (the current view only; a
// previous view is projected into unjittered)
void view_of(const dof_camera &c, const LensDerived &q, dof::ViewConst &v, bool jitter)
{
    memcpy(v.pos, c.pos, sizeof(v.pos));
    memcpy(v.right, c.right, sizeof(v.right));
    memcpy(v.up, c.up, sizeof(v.up));
    memcpy(v.fwd, c.fwd, sizeof(v.fwd));
    v.tanx = q.tanx;
    v.tany = q.tany;
    v.ju = jitter ? (c.jitter[0] * 2.0f) / (float)c.width : 0.0f;
    v.jv = jitter ? (c.jitter[1] * 2.0f) / (float)c.height : 0.0f;
}

// 81 taps: centre + rings k = 1..4 of 8k taps at radius k/4, angle 2 pi j / 8k
// (section 3.1.1), evaluated in binary64 then rounded.
// The gather's taps on the aperture polygon (pp_polygon): ring k holds 8k
// taps at equal arc length on the polygon of circumradius k/4 whose corners
// sit at rot + 2 pi i / B (between the blade normals), the first half a step
// past corner 0; ring distance k/4.  Offsets are the far-field image of the
// aperture on screen (lens up = screen -y) reflected for gathering: lens
// point (x, y) -> offset (-x, y).  Binary64 on the host, rounded once.
dof::Rings make_polygon_rings(int blades, float rot)
{
    dof::Rings r;
    r.ox[0] = 0.0f;
    r.oy[0] = 0.0f;
    r.frac[0] = 0.0f;
    const double pi = 3.14159265358979323846;
    const double side = 2.0 * sin(pi / blades);
    int i = 1;
    for (int k = 1; k <= 4; ++k) {
        const int taps = 8 * k;
        for (int j = 0; j < taps; ++j, ++i) {
            const double s = ((double)j + 0.5) * ((double)blades * side) / (double)taps;
            int e = (int)floor(s / side);
            if (e >= blades) e = blades - 1;
            const double u = s / side - (double)e;
            const double a0 = (double)rot + 2.0 * pi * e / blades, a1 = (double)rot + 2.0 * pi * (e + 1) / blades;
            const double px = (1.0 - u) * cos(a0) + u * cos(a1), py = (1.0 - u) * sin(a0) + u * sin(a1);
            r.ox[i] = (float)(k / 4.0 * -px);
            r.oy[i] = (float)(k / 4.0 * py);
            r.frac[i] = (float)k * 0.25f;
        }
    }
    return r;
}

dof::Rings make_rings()
{
    dof::Rings r;
    r.ox[0] = 0.0f;
    r.oy[0] = 0.0f;
    r.frac[0] = 0.0f;
    int i = 1;
    const double pi = 3.14159265358979323846;
    for (int k = 1; k <= 4; ++k) {
        const int taps = 8 * k;
        for (int j = 0; j < taps; ++j, ++i) {
            const double ang = 2.0 * pi * (double)j / (double)taps;
            r.ox[i] = (float)(k / 4.0 * cos(ang));
            r.oy[i] = (float)(k / 4.0 * sin(ang));
            r.frac[i] = (float)k * 0.25f;
        }
    }
    return r;
}

// Regular-polygon aperture: inward edge normals at blade_rot + pi/n + 2 pi i/n,
// apothem cos(pi / n) for a unit circumradius.
void make_aperture(const dof_lens &l, dof::Aperture &ap)
{
    memset(&ap, 0, sizeof(ap));
    ap.blades = l.blades;
    ap.apothem = 1.0f;
    if (l.blades >= 3) {
        const double pi = 3.14159265358979323846;
        const int n = l.blades;
        ap.apothem = (float)cos(pi / n);
        for (int i = 0; i < n; ++i) {
            const double th = (double)l.blade_rot + pi / n + 2.0 * pi * i / n;
            ap.nx[i] = (float)cos(th);
            ap.ny[i] = (float)sin(th);
        }
    }
}

bool lens_ok(const dof_lens *l)
{
    if (!l) return false;
    if (!(l->focal > 0.0f) || !(l->fnum > 0.0f) || !(l->sensor > 0.0f) || !(l->focus > l->focal)) return false;
    if (!(l->focal < INFINITY) || !(l->focus < INFINITY) || !(l->sensor < INFINITY)) return false;
    return l->blades == 0 || (l->blades >= 3 && l->blades <= dof::kMaxBlades);
}

bool camera_ok(const dof_camera *c)
{
    if (!c || c->width <= 0 || c->height <= 0 || (c->width & 1) || (c->height & 1)) return false;
    if ((int64_t)c->width * c->height > (int64_t)1 << 30) return false;
    for (int a = 0; a < 3; ++a)
        if (!isfinite(c->pos[a]) || !isfinite(c->right[a]) || !isfinite(c->up[a]) || !isfinite(c->fwd[a])) return false;
    if (!(fabsf(c->jitter[0]) <= 1.0f) || !(fabsf(c->jitter[1]) <= 1.0f)) return false;
    return true;
}

// Ray indices, counts and the traversal's work counter are 32-bit: a frame
// may ask for at most 2^31 rays (half-res pixels x m).
constexpr int64_t kMaxFrameRays = (int64_t)1 << 31;
bool rays_fit(int width, int height, int m) { return (int64_t)(width / 2) * (height / 2) * m <= kMaxFrameRays; }

dof_status params_check(const dof_params *p)
{
    if (!p) return fail(DOF_E_INVALID, "params is NULL");
    if (p->struct_size != sizeof(dof_params)) return fail(DOF_E_INVALID, "params.struct_size mismatch");
    if (p->m < 1 || p->m > 255) return fail(DOF_E_INVALID, "m must be in 1..255");
    if (p->tile != dof::kTile) return fail(DOF_E_UNSUPPORTED, "tile must be 16");
    if (p->mask_mode < 0 || p->mask_mode > 3) return fail(DOF_E_INVALID, "bad mask_mode");
    if (p->pp_polygon != 0 && p->pp_polygon != 1) return fail(DOF_E_INVALID, "bad pp_polygon");
    if (p->taa < 0 || p->taa > (DOF_TAA_FINAL | DOF_TAA_RASTER | DOF_TAA_POST)) return fail(DOF_E_INVALID, "bad taa");
    if (p->ray_records != 0 && p->ray_records != 1) return fail(DOF_E_INVALID, "bad ray_records");
    if (p->composite_literal != 0 && p->composite_literal != 1) return fail(DOF_E_INVALID, "bad composite_literal");
    if (p->gather_window != 0 && p->gather_window != -1 && p->gather_window != 32 && p->gather_window != 40 &&
        p->gather_window != 48)
        return fail(DOF_E_INVALID, "gather_window must be 0, -1, 32, 40 or 48");
    if (p->trace_stack != 0 && p->trace_stack != 16 && p->trace_stack != 24 && p->trace_stack != 32)
        return fail(DOF_E_INVALID, "trace_stack must be 0, 16, 24 or 32");
    if (p->trace_grab < 0 || p->trace_grab > 256 || p->trace_refill < 0 || p->trace_refill > 64 ||
        p->trace_leaf_batch < 0 || p->trace_leaf_batch > 64)
        return fail(DOF_E_INVALID, "trace_grab must be in 0..256, trace_refill and trace_leaf_batch in 0..64");
    if (p->trace_order < 0 || p->trace_order > 2) return fail(DOF_E_INVALID, "trace_order must be 0, 1 or 2");
    if (p->trace_steps != 0 && p->trace_steps != 3 && p->trace_steps != 4)
        return fail(DOF_E_INVALID, "trace_steps must be 0, 3 or 4");
    if (p->mask_mode == DOF_MASK_DILATE && p->r_max > 32.0f)
        return fail(DOF_E_UNSUPPORTED, "mask dilation supports r_max <= 32");
    if (!(p->r_max > 0.0f) || !(p->depth_range > 0.0f) || !(p->h_edge > 0.0f)) return fail(DOF_E_INVALID, "bad params");
    if (!(p->lod_max >= 0.0f)) return fail(DOF_E_INVALID, "bad lod_max");
    if (p->trace_blocks < 0 || p->trace_blocks > dof::kMaxTraceBlocks) return fail(DOF_E_INVALID, "bad trace_blocks");
    return DOF_OK;
}

dof::TraceKnobs trace_knobs(const dof_params &p)
{
    dof::TraceKnobs k;
    k.stack = p.trace_stack ? p.trace_stack : dof::kStackLds;
    k.grab = p.trace_grab ? (uint32_t)p.trace_grab : 64u;
    k.refill = p.trace_refill ? p.trace_refill : 16;
    k.leaf_batch = p.trace_leaf_batch ? p.trace_leaf_batch : 32;
    k.reverse = p.trace_order == 1 ? 0 : 1;
    k.steps = p.trace_steps ? p.trace_steps : dof::kTraceSteps;
    return k;
}

void fill_frame_const(const dof_scene *s, const dof_camera &cam, const dof_lens &lens, const dof_params &p,
                      bool have_hist, bool motion, const dof_camera &pcam, const dof_lens &plens,
                      dof::FrameConst &fc)
{
    memset(&fc, 0, sizeof(fc));
    const int W = cam.width, H = cam.height;
    fc.W = W;
    fc.H = H;
    fc.hw = W / 2;
    fc.hh = H / 2;
    fc.T = p.tile;
    fc.tw = (fc.hw + fc.T - 1) / fc.T;
    fc.th = (fc.hh + fc.T - 1) / fc.T;
    fc.D = (int)ceilf(p.r_max / (float)fc.T);
    fc.m = p.m;
    fc.mask_mode = p.mask_mode;
    fc.taa = p.taa;
    fc.ray_records = p.ray_records;
    fc.composite_literal = p.composite_literal;
    fc.gather_win = p.gather_window <= 0 ? 0 : p.gather_window;
    fc.tk = trace_knobs(p);
    fc.have_hist = have_hist;
    fc.motion = motion;
    fc.seed = cam.seed;
    fc.frame = cam.frame;
    const LensDerived q = lens_derived(lens, W, H);
    fc.d = lens.focus;
    fc.half_a = q.half_a;
    fc.cock = q.cock;
    fc.znb = q.znb;
    fc.ramp = q.ramp;
    fc.s = p.s;
    fc.var_mask_w = p.var_mask_w;
    fc.alpha_h = motion ? p.alpha_motion : p.alpha;
    fc.var_recon_w = p.var_recon_w;
    fc.b_max = p.b_max;
    fc.h_edge = p.h_edge;
    fc.lod_scale = p.lod_scale;
    fc.lod_max = p.lod_max;
    fc.lod_levels = p.lod_max >= 3.0f ? 3 : (int)p.lod_max;
    fc.depth_range = p.depth_range;
    fc.r_max = p.r_max;
    fc.l_spec = p.l_spec;
    view_of(cam, q, fc.cur, true);
    view_of(have_hist ? pcam : cam, have_hist ? lens_derived(plens, W, H) : q, fc.prev, false);
    make_aperture(lens, fc.ap);
    if (s) memcpy(&fc.shade, &s->shade, sizeof(fc.shade));
    int w = fc.hw, h = fc.hh;
    int64_t off = 0;
    for (int l = 0; l < 4; ++l) {
        fc.mw[l] = w;
        fc.mh[l] = h;
        fc.moff[l] = off;
        off += (int64_t)w * h;
        w = (w + 1) >> 1;
        h = (h + 1) >> 1;
    }
}

bool same_view(const dof_camera &a, const dof_camera &b, const dof_lens &la, const dof_lens &lb)
{
    return memcmp(a.pos, b.pos, sizeof(a.pos)) == 0 && memcmp(a.right, b.right, sizeof(a.right)) == 0 &&
           memcmp(a.up, b.up, sizeof(a.up)) == 0 && memcmp(a.fwd, b.fwd, sizeof(a.fwd)) == 0 &&
           memcmp(&la, &lb, sizeof(la)) == 0;
}

int default_trace_blocks(bool batch = false, int stack = dof::kStackLds, int steps = dof::kTraceSteps)
{
    // as many 128-thread blocks as fit on the device at once (registers and
    // the LDS stack decide), capped at the grid limit
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 1024;
    per_cu = dof::trace_blocks_per_cu(batch, stack, steps);
    if (per_cu <= 0) per_cu = 5;
    const int b = cus * per_cu;
    return b > dof::kMaxTraceBlocks ? dof::kMaxTraceBlocks : b;
}

// Checks of one frame's arguments (shared by single frames and batches);
// on success L is the frame's scratch layout and fc its constants.
dof_status check_frame(dof_scene *scene, const dof_camera *cam, const dof_lens *lens, const dof_gbuffer *gb,
                       const dof_history_io *hist, const dof_params *p, const dof_frame_out *out, void *scratch,
                       size_t scratch_bytes, dof::ScratchLayout &L, dof::FrameConst &fc, bool &have_hist)
{
    if (!scene) return fail(DOF_E_INVALID, "scene is NULL");
    if (!camera_ok(cam)) return fail(DOF_E_INVALID, "bad camera (even positive size, finite basis, |jitter| <= 1)");
    if (!lens_ok(lens)) return fail(DOF_E_INVALID, "bad lens");
    dof_status st = params_check(p);
    if (st != DOF_OK) return st;
    if (!gb || !gb->colour || !gb->depth || !gb->normal) return fail(DOF_E_INVALID, "bad G-buffer");
    if ((gb->colour_format != DOF_RGBA32F && gb->colour_format != DOF_RGBA16F) ||
        (gb->normal_format != DOF_RGBA32F && gb->normal_format != DOF_RGBA16F))
        return fail(DOF_E_INVALID, "bad G-buffer format");
    if (!hist || !hist->out) return fail(DOF_E_INVALID, "history output is NULL");
    if (hist->in && hist->in == hist->out) return fail(DOF_E_INVALID, "history in and out must differ");
    if (!out || !out->colour || !out->mask) return fail(DOF_E_INVALID, "bad frame output");
    if (out->colour_format != DOF_RGBA32F && out->colour_format != DOF_RGBA16F)
        return fail(DOF_E_INVALID, "bad output format");
    if (!scratch) return fail(DOF_E_INVALID, "scratch is NULL");
    if (!scene->built) return fail(DOF_E_STATE, "BVH not built");
    if (!rays_fit(cam->width, cam->height, p->m))
        return fail(DOF_E_UNSUPPORTED, "half-res pixels x m exceeds 2^31 rays per frame");
    L = frame_layout(cam->width, cam->height, p->m, p->taa, p->ray_records);
    if (scratch_bytes < L.total) return fail(DOF_E_NOMEM, "scratch needs %zu bytes, got %zu", L.total, scratch_bytes);
    have_hist = !hist->reset && hist->in && hist->prev_camera.width == cam->width &&
                hist->prev_camera.height == cam->height && lens_ok(&hist->prev_lens);
    const bool motion = have_hist && !same_view(*cam, hist->prev_camera, *lens, hist->prev_lens);
    fill_frame_const(scene, *cam, *lens, *p, have_hist, motion, hist->prev_camera, hist->prev_lens, fc);
    return DOF_OK;
}

// The ground-truth renderer traces at most this many rays per traversal
// launch (whole pixels); its scratch holds their 8-byte (leaf, t) records.
constexpr int64_t kRefChunkRays = (int64_t)1 << 22;
constexpr int kRefMaxSpp = 1024;

int64_t reference_chunk_px(int width, int height, int spp)
{
    const int64_t px = (int64_t)width * height;
    const int64_t c = kRefChunkRays / spp;
    return c < px ? (c < 1 ? 1 : c) : px;
}

const dof::Rings &ring_table()
{
    static const dof::Rings rings = make_rings();
    return rings;
}

// the post-process gather's kernel for a lens and parameters
dof::Rings gather_rings(const dof_lens &lens, const dof_params &p)
{
    return (p.pp_polygon && lens.blades >= 3) ? make_polygon_rings(lens.blades, lens.blade_rot) : ring_table();
}

}  // namespace

// A post-process chain's stream (non-blocking, default priority) with its
// fork and join events, on the current device; false when any of them could
// not be created (then nothing is left allocated).
static bool side_create(dof::SideStream &sd)
{
    if (hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking) != hipSuccess) return false;
    if (hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(sd.stream);
        return false;
    }
    if (hipEventCreateWithFlags(&sd.join, hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(sd.fork);
        (void)hipStreamDestroy(sd.stream);
        return false;
    }
    return true;
}

static void side_destroy(dof::SideStream &sd)
{
    (void)hipEventDestroy(sd.fork);
    (void)hipEventDestroy(sd.join);
    (void)hipStreamDestroy(sd.stream);
}

struct dof_batch {
    char *table;                       // device: BatchHead, then the jobs
    size_t table_bytes;
    int32_t max_items;
    int32_t n;                         // jobs of the current set (0 = none)
    uint32_t nblk[dof::kNumGrids];     // total blocks of each grid shape
    int32_t trace_blocks;
    bool dilate;                       // params.mask_mode == DOF_MASK_DILATE
    int64_t max_rays;                  // sum over the items of half-res pixels x m
    int taa;                           // params.taa (DOF_TAA_* bits)
    int gather_win;                    // the gather's LDS window (params.gather_window)
    dof::TraceKnobs tk;                // traversal launch knobs (params.trace_*)
    std::vector<char> host;            // staging copy of the table
    bool side_ready;                   // side holds a stream and two events
    dof::SideStream side;              // the post-process chain's stream
};

// the error message of a failing call made in another translation unit
dof_status dof::set_error(dof_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vfail(code, fmt, ap);
    va_end(ap);
    return code;
}

extern "C" {

int32_t dof_abi_version(void) { return DOF_ABI_VERSION; }

const char *dof_last_error(void) { return g_err; }

void dof_default_params(dof_params *p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(dof_params);
    p->m = 8;
    p->s = 0.8f;
    p->var_mask_w = 1.0e5f;
    p->alpha = 0.95f;
    p->alpha_motion = 0.8f;
    p->var_recon_w = 2000.0f;
    p->b_max = 0.9f;
    p->h_edge = 0.3f;
    p->lod_scale = 0.05f;
    p->lod_max = 3.0f;
    p->depth_range = 0.1f;
    p->r_max = 32.0f;
    p->tile = dof::kTile;
    p->l_spec = 1.0f;
    p->mask_mode = DOF_MASK_ADAPTIVE;
    p->trace_blocks = 0;
}

dof_status dof_scene_bytes(int32_t ntri, size_t *bytes)
{
    if (ntri <= 0 || !bytes) return fail(DOF_E_INVALID, "ntri must be > 0 and bytes non-NULL");
    *bytes = scene_layout(ntri, (int64_t)kMaxRefsPerTri * ntri).total;
    return DOF_OK;
}

static dof_status check_desc(const dof_scene_desc *desc)
{
    if (!desc || !desc->verts || !desc->albedo || desc->ntri <= 0)
        return fail(DOF_E_INVALID, "scene description: NULL argument or ntri <= 0");
    if (desc->leaf_split < 0 || desc->leaf_split > kMaxLeafSplit)
        return fail(DOF_E_INVALID, "leaf_split must be 0..%d", kMaxLeafSplit);
    return DOF_OK;
}

dof_status dof_scene_bytes_desc(const dof_scene_desc *desc, size_t *bytes)
{
    if (!bytes) return fail(DOF_E_INVALID, "bytes is NULL");
    const dof_status st = check_desc(desc);
    if (st != DOF_OK) return st;
    const int64_t n = leaf_refs(desc, nullptr);
    if (n < 0) return fail(DOF_E_UNSUPPORTED, "more than 2^31 - 1 leaf references");
    *bytes = scene_layout(desc->ntri, n).total;
    return DOF_OK;
}

dof_status dof_create_scene(const dof_scene_desc *desc, void *arena, size_t arena_bytes, void *stream,
                            dof_scene **out)
{
    if (!out || !arena) return fail(DOF_E_INVALID, "dof_create_scene: NULL argument");
    const dof_status st0 = check_desc(desc);
    if (st0 != DOF_OK) return st0;
    *out = nullptr;
    std::vector<uint32_t> ref_off;
    try {
        ref_off.resize((size_t)desc->ntri + 1);
    } catch (...) {
        return fail(DOF_E_NOMEM, "host allocation failed");
    }
    const int64_t nleaf = leaf_refs(desc, ref_off.data());
    if (nleaf < 0) return fail(DOF_E_UNSUPPORTED, "more than 2^31 - 1 leaf references");
    const SceneLayout L = scene_layout(desc->ntri, nleaf);
    if (arena_bytes < L.total) return fail(DOF_E_NOMEM, "scene arena needs %zu bytes, got %zu", L.total, arena_bytes);
    dof_scene *s = new (std::nothrow) dof_scene;
    if (!s) return fail(DOF_E_NOMEM, "host allocation failed");
    memset(s, 0, sizeof(*s));
    char *a = static_cast<char *>(arena);
    s->arena = a;
    s->arena_bytes = arena_bytes;
    dof::SceneDev &d = s->dev;
    d.ntri = desc->ntri;
    d.nleaf = (int32_t)nleaf;
    d.verts_in = reinterpret_cast<float *>(a + L.verts_in);
    d.albedo_in = reinterpret_cast<float *>(a + L.albedo_in);
    d.ref_off = reinterpret_cast<uint32_t *>(a + L.ref_off);
    d.ref_box = reinterpret_cast<float *>(a + L.ref_box);
    d.ref_tri = reinterpret_cast<uint32_t *>(a + L.ref_tri);
    d.tris = reinterpret_cast<float4 *>(a + L.tris);
    d.albedo = reinterpret_cast<float4 *>(a + L.albedo);
    d.nodes = reinterpret_cast<dof::BvhNode *>(a + L.nodes);
    d.nodes16 = reinterpret_cast<dof::BvhNode16 *>(a + L.nodes16);
    d.parent = reinterpret_cast<uint32_t *>(a + L.parent);
    d.keys = reinterpret_cast<uint64_t *>(a + L.keys);
    d.keys_tmp = reinterpret_cast<uint64_t *>(a + L.keys_tmp);
    d.ids = reinterpret_cast<uint32_t *>(a + L.ids);
    d.ids_tmp = reinterpret_cast<uint32_t *>(a + L.ids_tmp);
    d.flags = reinterpret_cast<uint32_t *>(a + L.flags);
    d.hist = reinterpret_cast<uint32_t *>(a + L.hist);
    d.bounds = reinterpret_cast<float *>(a + L.bounds);
    d.aux = reinterpret_cast<uint32_t *>(a + L.aux);
    d.sort_blocks = L.sort_blocks;
    d.bound_blocks = L.bound_blocks;
    memcpy(s->shade.light_dir, desc->light_dir, sizeof(desc->light_dir));
    memcpy(s->shade.light_rad, desc->light_rad, sizeof(desc->light_rad));
    memcpy(s->shade.ambient, desc->ambient, sizeof(desc->ambient));
    memcpy(s->shade.sky, desc->sky, sizeof(desc->sky));
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(a + L.verts_in, desc->verts, sizeof(float) * 9 * (size_t)desc->ntri,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(a + L.albedo_in, desc->albedo, sizeof(float) * 3 * (size_t)desc->ntri,
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(a + L.ref_off, ref_off.data(), sizeof(uint32_t) * ref_off.size(), hipMemcpyHostToDevice,
                           st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete s;
        return fail(DOF_E_DEVICE, "scene upload: %s", hipGetErrorString(e));
    }
    // the post-process chain's stream and its fork / join events; without
    // them frames run on the caller's stream alone
    s->side_ready = side_create(s->side);
    *out = s;
    return DOF_OK;
}

dof_status dof_build_bvh(dof_scene *scene, void *stream)
{
    const Range range("dof_build_bvh");
    if (!scene) return fail(DOF_E_INVALID, "scene is NULL");
    DOF_HIP(dof::launch_build_bvh(scene->dev, static_cast<hipStream_t>(stream)));
    scene->built = true;
    return DOF_OK;
}

dof_status dof_bvh_view_get(const dof_scene *scene, dof_bvh_view *out)
{
    if (!scene || !out) return fail(DOF_E_INVALID, "NULL argument");
    if (!scene->built) return fail(DOF_E_STATE, "BVH not built");
    out->ntri = scene->dev.ntri;
    out->nleaf = scene->dev.nleaf;
    out->keys = scene->dev.keys;
    out->ids = scene->dev.ids;
    out->parent = scene->dev.parent;
    out->nodes = scene->dev.nodes;
    out->nodes16 = scene->dev.nodes16;
    out->tris = scene->dev.tris;
    return DOF_OK;
}

void dof_destroy_scene(dof_scene *scene)
{
    if (!scene) return;
    if (scene->events_ready)
        for (int i = 0; i <= DOF_NUM_STAGES; ++i) (void)hipEventDestroy(scene->ev[i]);
    if (scene->side_ready) side_destroy(scene->side);
    delete scene;
}

dof_status dof_trace_rays(const dof_scene *scene, int64_t n, const float *org, const float *dir, int32_t *hit,
                          float *t, void *stream)
{
    if (!scene || n < 0 || (n > 0 && (!org || !dir || !hit || !t))) return fail(DOF_E_INVALID, "bad arguments");
    if (!scene->built) return fail(DOF_E_STATE, "BVH not built");
    if (n > ((int64_t)1 << 31)) return fail(DOF_E_INVALID, "too many rays");
    DOF_HIP(dof::launch_trace_rays(scene->dev, n, org, dir, hit, t, default_trace_blocks(),
                                   static_cast<hipStream_t>(stream)));
    return DOF_OK;
}

dof_status dof_render_gbuffer(const dof_scene *scene, const dof_camera *cam, const dof_lens *lens, void *colour,
                              int32_t colour_format, float *depth, void *normal, int32_t normal_format, void *stream)
{
    if (!scene || !camera_ok(cam) || !lens_ok(lens) || !colour || !depth || !normal)
        return fail(DOF_E_INVALID, "dof_render_gbuffer: bad arguments");
    if ((colour_format != DOF_RGBA32F && colour_format != DOF_RGBA16F) ||
        (normal_format != DOF_RGBA32F && normal_format != DOF_RGBA16F))
        return fail(DOF_E_INVALID, "bad format");
    if (!scene->built) return fail(DOF_E_STATE, "BVH not built");
    dof_params p;
    dof_default_params(&p);
    dof::FrameConst fc;
    fill_frame_const(scene, *cam, *lens, p, false, false, *cam, *lens, fc);
    DOF_HIP(dof::launch_gbuffer(scene->dev, fc, colour, colour_format, depth, normal, normal_format,
                                default_trace_blocks(), static_cast<hipStream_t>(stream)));
    return DOF_OK;
}

dof_status dof_reference_scratch_bytes(int32_t width, int32_t height, int32_t spp, size_t *bytes)
{
    if (width <= 0 || height <= 0 || (width & 1) || (height & 1) || !bytes)
        return fail(DOF_E_INVALID, "width/height must be even and positive");
    if ((int64_t)width * height > (int64_t)1 << 30) return fail(DOF_E_INVALID, "image too large");
    if (spp < 1 || spp > kRefMaxSpp) return fail(DOF_E_INVALID, "spp must be in 1..%d", kRefMaxSpp);
    *bytes = sizeof(uint2) * (size_t)(reference_chunk_px(width, height, spp) * spp);
    return DOF_OK;
}

dof_status dof_render_reference(dof_scene *scene, const dof_camera *cam, const dof_lens *lens, int32_t spp,
                                void *colour, int32_t colour_format, void *scratch, size_t scratch_bytes, void *stream)
{
    const Range range("dof_render_reference");
    if (!scene || !camera_ok(cam) || !lens_ok(lens) || !colour || !scratch)
        return fail(DOF_E_INVALID, "dof_render_reference: bad arguments");
    if (colour_format != DOF_RGBA32F && colour_format != DOF_RGBA16F) return fail(DOF_E_INVALID, "bad format");
    size_t need = 0;
    dof_status st = dof_reference_scratch_bytes(cam->width, cam->height, spp, &need);
    if (st != DOF_OK) return st;
    if (scratch_bytes < need) return fail(DOF_E_NOMEM, "scratch needs %zu bytes, got %zu", need, scratch_bytes);
    if (!scene->built) return fail(DOF_E_STATE, "BVH not built");
    dof_params p;
    dof_default_params(&p);
    dof::FrameConst fc;
    fill_frame_const(scene, *cam, *lens, p, false, false, *cam, *lens, fc);
    DOF_HIP(dof::launch_reference(scene->dev, fc, spp, static_cast<uint2 *>(scratch),
                                  reference_chunk_px(cam->width, cam->height, spp), colour, colour_format,
                                  default_trace_blocks(), static_cast<hipStream_t>(stream)));
    return DOF_OK;
}

dof_status dof_history_bytes(int32_t width, int32_t height, size_t *bytes)
{
    if (width <= 0 || height <= 0 || (width & 1) || (height & 1) || !bytes)
        return fail(DOF_E_INVALID, "width/height must be even and positive");
    const size_t record = ((size_t)(width / 2) * (height / 2) * 52 + 15) & ~(size_t)15;
    // the half-res record, then the TAA planes: final and raster (full res), post-filter (half res)
    *bytes = record + (size_t)width * height * 32 + (size_t)(width / 2) * (height / 2) * 16;
    return DOF_OK;
}

dof_status dof_history_reset(void *hist, int32_t width, int32_t height, void *stream)
{
    size_t b = 0;
    dof_status st = dof_history_bytes(width, height, &b);
    if (st != DOF_OK) return st;
    if (!hist) return fail(DOF_E_INVALID, "hist is NULL");
    DOF_HIP(dof::launch_history_reset(static_cast<float *>(hist), (int64_t)(b / 4), static_cast<hipStream_t>(stream)));
    return DOF_OK;
}

dof_status dof_frame_scratch_bytes(int32_t width, int32_t height, const dof_params *p, size_t *bytes)
{
    if (width <= 0 || height <= 0 || (width & 1) || (height & 1) || !bytes)
        return fail(DOF_E_INVALID, "width/height must be even and positive");
    dof_status st = params_check(p);
    if (st != DOF_OK) return st;
    if (!rays_fit(width, height, p->m)) return fail(DOF_E_UNSUPPORTED, "half-res pixels x m exceeds 2^31 rays per frame");
    *bytes = frame_layout(width, height, p->m, p->taa, p->ray_records).total;
    return DOF_OK;
}

dof_status dof_render_frame(dof_scene *scene, const dof_camera *cam, const dof_lens *lens, const dof_gbuffer *gb,
                            const dof_history_io *hist, const dof_params *p, const dof_frame_out *out, void *scratch,
                            size_t scratch_bytes, void *stream)
{
    const Range range("dof_render_frame");
    dof::ScratchLayout L;
    dof::FrameConst fc;
    bool have_hist = false;
    dof_status st = check_frame(scene, cam, lens, gb, hist, p, out, scratch, scratch_bytes, L, fc, have_hist);
    if (st != DOF_OK) return st;
    const dof::Rings &rings = ring_table();
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *scr = static_cast<char *>(scratch);
    const void *hin = have_hist ? hist->in : nullptr;
    hipEvent_t *ev = nullptr;
    if (p->timing) {
        if (!scene->events_ready) {
            for (int i = 0; i <= DOF_NUM_STAGES; ++i) DOF_HIP(hipEventCreate(&scene->ev[i]));
            scene->events_ready = true;
        }
        ev = scene->ev;
    }
    const dof::SideStream *side = (ev == nullptr && scene->side_ready) ? &scene->side : nullptr;
    DOF_HIP(dof::launch_frame_pre(fc, gather_rings(*lens, *p), L, scr, *gb, hin, hist->out, out->mask, ev, side, s));
    const int blocks = p->trace_blocks > 0 ? p->trace_blocks : default_trace_blocks(false, fc.tk.stack, fc.tk.steps);
    DOF_HIP(dof::launch_trace(scene->dev, fc, L, scr, blocks, s));
    DOF_HIP(dof::launch_frame_post(scene->dev, fc, rings, L, scr, *gb, hin, hist->out, out->mask, *out, ev, side, s));
    scene->timed_frame = ev != nullptr;
    return DOF_OK;
}

dof_status dof_batch_bytes(int32_t max_items, size_t *bytes)
{
    if (max_items < 1 || max_items > DOF_MAX_BATCH || !bytes) return fail(DOF_E_INVALID, "bad arguments");
    *bytes = dof::batch_table_bytes(max_items);
    return DOF_OK;
}

dof_status dof_batch_create(void *table, size_t table_bytes, int32_t max_items, dof_batch **out)
{
    if (!table || !out || max_items < 1 || max_items > DOF_MAX_BATCH) return fail(DOF_E_INVALID, "bad arguments");
    if ((reinterpret_cast<uintptr_t>(table) & 255u) != 0) return fail(DOF_E_INVALID, "table must be 256-byte aligned");
    if (table_bytes < dof::batch_table_bytes(max_items))
        return fail(DOF_E_NOMEM, "batch table needs %zu bytes, got %zu", dof::batch_table_bytes(max_items), table_bytes);
    dof_batch *b = new (std::nothrow) dof_batch();
    if (!b) return fail(DOF_E_NOMEM, "host allocation failed");
    b->table = static_cast<char *>(table);
    b->table_bytes = table_bytes;
    b->max_items = max_items;
    b->n = 0;
    b->side_ready = side_create(b->side);
    *out = b;
    return DOF_OK;
}

dof_status dof_batch_set(dof_batch *b, const dof_batch_item *items, int32_t n, const dof_params *p, void *stream)
{
    if (!b || !items || n < 1) return fail(DOF_E_INVALID, "bad arguments");
    if (n > b->max_items) return fail(DOF_E_NOMEM, "batch holds at most %d items, got %d", b->max_items, n);
    b->n = 0;
    const size_t jobs_at = dof::batch_table_bytes(0);
    b->host.assign(dof::batch_table_bytes(n), 0);
    dof::BatchHead *head = reinterpret_cast<dof::BatchHead *>(b->host.data());
    dof::Job *jobs = reinterpret_cast<dof::Job *>(b->host.data() + jobs_at);
    head->njobs = n;
    uint32_t tot[dof::kNumGrids] = {};
    int64_t max_rays = 0;
    for (int i = 0; i < n; ++i) {
        const dof_batch_item &it = items[i];
        dof::ScratchLayout L;
        dof::Job &J = jobs[i];
        bool have_hist = false;
        dof_status st = check_frame(it.scene, &it.camera, &it.lens, &it.gbuffer, &it.history, p, &it.out, it.scratch,
                                    it.scratch_bytes, L, J.fc, have_hist);
        if (st != DOF_OK) {
            char msg[sizeof(g_err)];
            snprintf(msg, sizeof(msg), "%s", g_err);
            return fail(st, "item %d: %s", i, msg);
        }
        for (int k = 0; k < i; ++k)
            if (items[k].scratch == it.scratch || items[k].history.out == it.history.out ||
                items[k].out.colour == it.out.colour)
                return fail(DOF_E_INVALID, "items %d and %d share a scratch, history output or colour buffer", k, i);
        char *scr = static_cast<char *>(it.scratch);
        J.P = dof::planes(J.fc, L, scr);
        J.gb_in = it.gbuffer;
        J.gb = dof::resolved_gbuffer(J.fc, J.P, it.gbuffer);
        J.hist_in = have_hist ? it.history.in : nullptr;
        J.hist_out = it.history.out;
        J.mask = it.out.mask;
        J.out = it.out;
        J.scene = dof::SceneArgs{it.scene->dev.nleaf, it.scene->dev.tris, it.scene->dev.albedo, it.scene->dev.nodes16,
                                 it.scene->dev.parent};
        J.grings = gather_rings(it.lens, *p);
        const dof::FrameConst &fc = J.fc;
        const int64_t np = (int64_t)fc.hw * fc.hh;
        max_rays += np * fc.m;
        if (max_rays > kMaxFrameRays) return fail(DOF_E_UNSUPPORTED, "batch exceeds 2^31 rays");
        auto cdiv = [](int64_t a, int64_t c) { return (uint32_t)((a + c - 1) / c); };
        const uint32_t bxs[dof::kNumGrids] = {(uint32_t)fc.tw, cdiv(fc.tw, 16), cdiv(fc.hw, 64), (uint32_t)L.nchunks,
                                              cdiv(np, 64), cdiv(fc.hw, 8), cdiv(fc.W, 64)};
        const uint32_t bys[dof::kNumGrids] = {(uint32_t)fc.th, cdiv(fc.th, 16), cdiv(fc.hh, 4), 1u, 1u,
                                              cdiv(fc.hh, 8), cdiv(fc.H, 4)};
        for (int g = 0; g < dof::kNumGrids; ++g) {
            J.bstart[g] = tot[g];
            J.bx[g] = bxs[g];
            const uint64_t t = (uint64_t)tot[g] + (uint64_t)bxs[g] * bys[g];
            if (t > 0x7fffffffu) return fail(DOF_E_INVALID, "batch too large for one launch");
            tot[g] = (uint32_t)t;
        }
    }
    DOF_HIP(hipMemcpyAsync(b->table, b->host.data(), b->host.size(), hipMemcpyHostToDevice,
                           static_cast<hipStream_t>(stream)));
    for (int g = 0; g < dof::kNumGrids; ++g) b->nblk[g] = tot[g];
    b->trace_blocks = p->trace_blocks > 0 ? p->trace_blocks : default_trace_blocks(true, jobs[0].fc.tk.stack, jobs[0].fc.tk.steps);
    b->dilate = p->mask_mode == DOF_MASK_DILATE;
    b->taa = p->taa;
    b->gather_win = jobs[0].fc.gather_win;
    b->tk = jobs[0].fc.tk;
    b->max_rays = max_rays;
    b->n = n;
    return DOF_OK;
}

dof_status dof_batch_run(dof_batch *b, dof_batch_stats *stats, void *stream)
{
    const Range range("dof_batch_run");
    if (!b) return fail(DOF_E_INVALID, "batch is NULL");
    if (b->n < 1) return fail(DOF_E_STATE, "no items set");
    hipStream_t s = static_cast<hipStream_t>(stream);
    dof::BatchHead *head = reinterpret_cast<dof::BatchHead *>(b->table);
    const dof::Job *jobs = reinterpret_cast<const dof::Job *>(b->table + dof::batch_table_bytes(0));
    const dof::Rings &rings = ring_table();
    // as for a frame, the post-process chain runs on the batch's side stream
    // beside the traversal, forked after the ray generation
    const dof::SideStream *side = b->side_ready ? &b->side : nullptr;
    DOF_HIP(dof::launch_batch_pre(head, jobs, b->n, b->nblk, rings, b->dilate, b->taa, b->gather_win, side, s));
    DOF_HIP(dof::launch_batch_raygen(head, jobs, b->n, b->max_rays, s));
    if (side) {
        DOF_HIP(hipEventRecord(side->fork, s));
        DOF_HIP(hipStreamWaitEvent(side->stream, side->fork, 0));
        DOF_HIP(dof::launch_batch_chain(jobs, b->n, b->nblk, rings, !b->dilate, b->taa, b->gather_win, side->stream));
        DOF_HIP(hipEventRecord(side->join, side->stream));
    }
    DOF_HIP(dof::launch_batch_trace(head, jobs, b->n, b->trace_blocks, b->tk, s));
    DOF_HIP(dof::launch_batch_post(head, jobs, b->n, b->nblk, rings, b->taa, side, s));
    if (stats) DOF_HIP(hipMemcpyAsync(stats, b->table, sizeof(dof_batch_stats), hipMemcpyDeviceToDevice, s));
    return DOF_OK;
}

void dof_batch_destroy(dof_batch *b)
{
    if (!b) return;
    if (b->side_ready) side_destroy(b->side);
    delete b;
}

dof_status dof_stage_times(dof_scene *scene, float *ms, int32_t cap, int32_t *n)
{
    if (!scene || !ms || cap < 0 || !n) return fail(DOF_E_INVALID, "bad arguments");
    if (!scene->timed_frame) return fail(DOF_E_STATE, "no frame rendered with params.timing set");
    DOF_HIP(hipEventSynchronize(scene->ev[DOF_NUM_STAGES]));
    const int k = cap < DOF_NUM_STAGES ? cap : DOF_NUM_STAGES;
    for (int i = 0; i < k; ++i) DOF_HIP(hipEventElapsedTime(&ms[i], scene->ev[i], scene->ev[i + 1]));
    *n = k;
    return DOF_OK;
}

dof_status dof_debug_view_get(void *scratch, int32_t width, int32_t height, const dof_params *p, dof_debug_view *out)
{
    if (!scratch || !out || width <= 0 || height <= 0 || (width & 1) || (height & 1))
        return fail(DOF_E_INVALID, "bad arguments");
    dof_status st = params_check(p);
    if (st != DOF_OK) return st;
    const dof::ScratchLayout L = frame_layout(width, height, p->m, p->taa, p->ray_records);
    char *s = static_cast<char *>(scratch);
    out->colr = s + L.colr;
    out->zn = s + L.zn;
    out->tile_max = s + L.tile_max;
    out->tile_dil = s + L.tile_dil;
    out->pre = s + L.pre;
    out->gather = s + L.gather;
    out->ppmed = s + L.ppmed;
    out->prev_idx = s + L.prev_idx;
    out->queue = s + L.queue;
    out->ray_base = s + L.ray_base;
    const bool rec = p->ray_records != 0;
    out->ray_hit = rec ? s + L.ray_hit : nullptr;
    out->ray_t = rec ? s + L.ray_t : nullptr;
    out->ray_col = rec ? s + L.ray_col : nullptr;
    out->ray_pos = rec ? s + L.ray_pos : nullptr;
    out->resolve = s + L.resolve;
    out->temporal = s + L.temporal;
    out->var_blur = s + L.var_blur;
    out->rtmed = s + L.rtmed;
    out->mips = s + L.mips;
    out->recon = s + L.recon;
    out->counters = s + L.counters;
    return DOF_OK;
}

}  // extern "C"
