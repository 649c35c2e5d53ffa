"""Oracle pins: Morton keys, the binary radix tree and closest-hit queries.

The paper traced against a DXR acceleration structure (section 4.1, timed in
the Ray Trace row of Table 2); the GPU path replaces it by an LBVH, so what is
pinned here is the definition of that tree and that the closest hit it finds
equals brute force over all triangles."""

import json
import math
import os

import numpy as np
import pytest

from paper_2210_06158_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LEAF = np.uint32(0x80000000)


def test_morton_golden(orc):
    g = json.load(open(os.path.join(GOLD, "morton_cases.json")))
    pts = np.array(g["points"], np.float32)
    verts = np.tile(pts, (1, 3))
    sc = orc.OracleScene(synth.Scene(verts, np.ones((len(pts), 3), np.float32)))
    assert orc.morton(sc).tolist() == g["codes"]
    # cubic cells and the large-triangle flag
    tv = np.array(g["triangles"], np.float32)
    sc = orc.OracleScene(synth.Scene(tv, np.ones((len(tv), 3), np.float32)))
    assert orc.morton(sc).tolist() == g["triangle_codes"]


def _tree_checks(codes, refs, left, right, parent, bounds, leaf_bounds, ref_boxes):
    """Checks of a binary radix tree over the 96-bit keys code << 32 | ref
    whose leaves are the references with boxes ref_boxes[ref]."""
    n = codes.size
    keys = [(int(c) << 32) | int(i) for c, i in zip(codes, refs)]
    refs = refs.astype(np.int64)
    assert all(a < b for a, b in zip(keys, keys[1:]))
    assert sorted(refs.tolist()) == list(range(n))
    assert np.array_equal(leaf_bounds, ref_boxes[refs])
    if n == 1:
        return
    seen_leaf = np.zeros(n, int)
    seen_node = np.zeros(n - 1, int)
    for ch in np.concatenate([left, right]):
        if ch & LEAF:
            seen_leaf[ch & ~LEAF] += 1
        else:
            seen_node[ch] += 1
    assert (seen_leaf == 1).all()
    assert seen_node[0] == 0 and (seen_node[1:] == 1).all()
    # ranges by explicit DFS, then the defining properties of each split
    stack = [(0, 0, n - 1)]
    while stack:
        node, f, l = stack.pop()
        assert node in (f, l)                        # one end carries the index
        diff = keys[f] ^ keys[l]
        b = diff.bit_length() - 1
        lc, rc = int(left[node]), int(right[node])
        split = (lc & 0x7FFFFFFF) if lc & 0x80000000 else lc
        ks = keys[f:l + 1]
        assert all(((k >> b) & 1) == 0 for k in ks[:split - f + 1])
        assert all(((k >> b) & 1) == 1 for k in ks[split - f + 1:])
        assert all((k >> (b + 1)) == (keys[f] >> (b + 1)) for k in ks)
        if rc & 0x80000000:
            assert (rc & 0x7FFFFFFF) == split + 1 == l
        else:
            assert rc == split + 1
        sub = ref_boxes[refs[f:l + 1]]
        assert np.array_equal(bounds[node], np.concatenate([sub[:, :3].min(0), sub[:, 3:].max(0)]))
        if lc & 0x80000000:
            assert split == f
            assert parent[n - 1 + split] == node
        else:
            assert parent[lc] == node
            stack.append((lc, f, split))
        if not rc & 0x80000000:
            assert parent[rc] == node
            stack.append((rc, split + 1, l))
        else:
            assert parent[n - 1 + l] == node


def _check_built_tree(orc, sc, v):
    b = sc.build_bvh()
    off, boxes, tri = sc.leaf_refs()
    n = boxes.shape[0]
    codes = orc.morton_boxes(boxes)
    assert np.array_equal(b["keys"], codes[b["refs"]])
    assert np.array_equal(b["ids"], tri[b["refs"]])
    # the references of each triangle, in order; an unsplit one is the triangle's box
    tv = v.reshape(-1, 3, 3)
    for i in range(tv.shape[0]):
        r = np.arange(off[i], off[i + 1])
        assert (tri[r] == i).all() and len(r) in (1, 4)
        if len(r) == 1:
            assert np.array_equal(boxes[r[0]], np.concatenate([tv[i].min(0), tv[i].max(0)]))
    _tree_checks(b["keys"], b["refs"], b["left"][:n - 1], b["right"][:n - 1], b["parent"], b["bounds"][:n - 1],
                 b["leaf_bounds"], boxes)
    return b, off, boxes, tri


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 513, 2000])
def test_radix_tree_properties(orc, n):
    v, a = synth.random_triangles(n, seed=100 + n)
    _check_built_tree(orc, orc.OracleScene(synth.Scene(v, a)), v)


def test_radix_tree_without_leaf_split_is_over_triangles(orc):
    v, a = synth.random_triangles(300, seed=9)
    sc = orc.OracleScene(synth.Scene(v, a), leaf_split=0)
    b, off, boxes, tri = _check_built_tree(orc, sc, v)
    assert np.array_equal(off, np.arange(301)) and np.array_equal(b["refs"], b["ids"])
    assert np.array_equal(b["keys"], orc.morton(sc)[b["ids"]])


def test_radix_tree_duplicate_codes(orc):
    # many coincident triangles share one Morton code; the reference index breaks ties
    v, a = synth.random_triangles(40, seed=5)
    v = np.concatenate([v, np.repeat(v[:3], 50, axis=0)])
    a = np.concatenate([a, np.repeat(a[:3], 50, axis=0)])
    _check_built_tree(orc, orc.OracleScene(synth.Scene(v, a)), v)


# ---------------------------------------------------------------- leaf references

def _exact_piece_box(tri, k, s0, s1):
    """Bounds of triangle tri (3x3, binary64) clipped to s0 <= x_k <= s1:
    Sutherland-Hodgman against both planes, then min / max."""
    def clip(poly, val, keep_ge):
        out = []
        for i in range(len(poly)):
            a, b = poly[i], poly[(i + 1) % len(poly)]
            ina = a[k] >= val if keep_ge else a[k] <= val
            inb = b[k] >= val if keep_ge else b[k] <= val
            if ina:
                out.append(a)
            if ina != inb:
                out.append(a + (b - a) * ((val - a[k]) / (b[k] - a[k])))
        return out
    poly = clip(clip([p for p in tri], s0, True), s1, False)
    pts = np.array(poly)
    return pts.min(0), pts.max(0)


def test_leaf_split_rule(orc):
    """Four references iff the box's three face areas sum to more than 8 times
    the triangle's area; the slabs cut the longest box axis in quarters."""
    g = json.load(open(os.path.join(GOLD, "leaf_split_cases.json")))
    for case in g["cases"]:
        v = np.array([case["verts"]], np.float32)
        sc = orc.OracleScene(synth.Scene(v, np.ones((1, 3), np.float32)))
        off, boxes, tri = sc.leaf_refs()
        assert int(off[1]) == case["refs"], case["name"]
        for box, want in zip(boxes, case.get("pieces", [])):
            lo, hi = np.array(want[:3]), np.array(want[3:])
            # the exact piece bounds lie inside, and the box exceeds them by at most 2^-18 of the scale
            assert (box[:3] <= lo).all() and (box[3:] >= hi).all(), case["name"]
            assert (lo - box[:3] <= 2.0 ** -18 * case["scale"]).all(), case["name"]
            assert (box[3:] - hi <= 2.0 ** -18 * case["scale"]).all(), case["name"]


@pytest.mark.parametrize("split,seed", [(1, 11), (2, 12), (3, 13)])
def test_leaf_split_pieces_cover_and_fit_the_triangle(orc, split, seed):
    """Each split triangle: its 2^split pieces' slabs tile its box along the
    longest axis, every piece box contains the exactly clipped piece
    (binary64) and exceeds it by at most 2^-18 of the triangle's size, and
    sample points of the triangle (including its vertices) lie in some piece
    box."""
    v, a = synth.random_triangles(400, seed=seed, size=1.5)
    sc = orc.OracleScene(synth.Scene(v, a), leaf_split=split)
    off, boxes, tri = sc.leaf_refs()
    tv = v.reshape(-1, 3, 3).astype(np.float64)
    nsplit = 0
    rng = np.random.default_rng(seed)
    for i in range(tv.shape[0]):
        r = np.arange(off[i], off[i + 1])
        if len(r) == 1:
            continue
        assert len(r) == 1 << split
        nsplit += 1
        lo, hi = tv[i].min(0), tv[i].max(0)
        ext = (hi - lo).astype(np.float32)
        k = int(np.argmax(ext))
        pb = boxes[r].astype(np.float64)
        assert pb[0, k] == lo[k] and pb[-1, 3 + k] == hi[k]
        assert (pb[1:, k] == pb[:-1, 3 + k]).all() and (pb[:, k] <= pb[:, 3 + k]).all()
        scale = float(np.abs(tv[i]).max() + (hi - lo).max())
        for j in range(len(r)):
            elo, ehi = _exact_piece_box(tv[i], k, pb[j, k], pb[j, 3 + k])
            assert (pb[j, :3] <= elo + 1e-12 * scale).all() and (pb[j, 3:] >= ehi - 1e-12 * scale).all()
            assert (elo - pb[j, :3] <= 2.0 ** -18 * scale).all() and (pb[j, 3:] - ehi <= 2.0 ** -18 * scale).all()
        w = rng.dirichlet([1, 1, 1], 200)
        pts = np.concatenate([w @ tv[i], tv[i]])
        for p in pts:
            inside = ((pb[:, :3] <= p) & (p <= pb[:, 3:])).all(1)
            assert inside.any()
    assert nsplit > 40


def test_leaf_split_keeps_every_closest_hit(orc):
    """Random soups with many thin triangles: the tree over split references
    finds the same closest hits as the tree over whole triangles, bit for bit."""
    v, a = synth.random_triangles(600, seed=21, size=1.2)
    o, d = _random_rays(3000, seed=22)
    s0 = orc.OracleScene(synth.Scene(v, a), leaf_split=0)
    h0, t0 = orc.closest_hit(s0, o, d)
    counts = [s0.leaf_refs()[0][-1]]
    for split in (1, 2, 3):
        s1 = orc.OracleScene(synth.Scene(v, a), leaf_split=split)
        h1, t1 = orc.closest_hit(s1, o, d)
        counts.append(s1.leaf_refs()[0][-1])
        assert np.array_equal(h1, h0) and np.array_equal(t1.view(np.uint32), t0.view(np.uint32))
    assert counts == sorted(counts) and counts[0] < counts[1]



@pytest.mark.parametrize("split", [0, 1, 2, 3])
def test_leaf_split_awkward_soup_equals_brute_force(orc, split):
    """Thin triangles at three coordinate scales up to 3e6, a vertex on a
    slab plane, a tie for the longest axis and degenerate triangles: every
    reference box holds its piece of the triangle and the tree's closest hits
    equal brute force over the triangles, bit for bit."""
    v, a, o, d = synth.awkward_triangles(4242)
    sc = orc.OracleScene(synth.Scene(v, a), leaf_split=split)
    off, boxes, tri = sc.leaf_refs()
    assert len(tri) == off[-1] and (split == 0) == (len(tri) == v.shape[0])
    tv = v.reshape(-1, 3, 3).astype(np.float64)
    lo, hi = tv.min(1), tv.max(1)
    assert np.all(boxes[:, :3] >= lo[tri]) and np.all(boxes[:, 3:] <= hi[tri])
    hb, tb = orc.closest_hit(sc, o, d, use_bvh=True)
    hf, tf = orc.closest_hit(sc, o, d, use_bvh=False)
    assert (hf >= 0).mean() > 0.3
    assert np.array_equal(hb, hf) and np.array_equal(tb.view(np.uint32), tf.view(np.uint32))

def _random_rays(n, seed, spread=5.0):
    rng = synth.SplitMix64(seed)
    o = rng.uniform(3 * n, -spread, spread).reshape(n, 3)
    tgt = rng.uniform(3 * n, -spread * 0.6, spread * 0.6).reshape(n, 3)
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


@pytest.mark.parametrize("n", [1, 2, 3, 50, 500, 3000])
def test_bvh_closest_hit_equals_brute_force(orc, n):
    v, a = synth.random_triangles(n, seed=300 + n, spread=4.0, size=0.8)
    sc = orc.OracleScene(synth.Scene(v, a))
    o, d = _random_rays(4000, seed=n)
    hb, tb = orc.closest_hit(sc, o, d, use_bvh=True)
    hf, tf = orc.closest_hit(sc, o, d, use_bvh=False)
    assert np.array_equal(hb, hf)
    assert np.array_equal(tb.view(np.uint32), tf.view(np.uint32))
    assert (hb >= 0).any()


def moller_trumbore(o, d, tri):
    """Closest hit in binary64 (Moller & Trumbore 1997), all rays x all
    triangles; returns (t, id, second-best t, min barycentric margin)."""
    o = o.astype(np.float64)[:, None, :]
    d = d.astype(np.float64)[:, None, :]
    v0, v1, v2 = (tri[:, i, :].astype(np.float64)[None] for i in range(3))
    e1, e2 = v1 - v0, v2 - v0
    p = np.cross(d, e2)
    det = (e1 * p).sum(-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        s = o - v0
        u = (s * p).sum(-1) * inv
        qv = np.cross(s, e1)
        w = (d * qv).sum(-1) * inv
        t = (e2 * qv).sum(-1) * inv
    ok = (np.abs(det) > 1e-12) & (u >= 0) & (w >= 0) & (u + w <= 1) & (t > 0)
    t = np.where(ok, t, np.inf)
    margin = np.where(ok, np.minimum(np.minimum(u, w), 1 - u - w), np.inf)
    order = np.argsort(t, axis=1)
    best = order[:, 0]
    rows = np.arange(t.shape[0])
    return t[rows, best], best, t[rows, order[:, 1]] if t.shape[1] > 1 else np.full(t.shape[0], np.inf), \
        margin[rows, best]


def test_closest_hit_matches_binary64_reference(orc):
    n = 300
    v, a = synth.random_triangles(n, seed=77, spread=3.0, size=0.7)
    sc = orc.OracleScene(synth.Scene(v, a))
    o, d = _random_rays(3000, seed=78)
    h, t = orc.closest_hit(sc, o, d)
    rt, rid, rt2, marg = moller_trumbore(o, d, v.reshape(-1, 3, 3))
    hit = np.isfinite(rt)
    clear = hit & (marg > 1e-4) & (rt2 > rt * (1 + 1e-4))
    assert clear.sum() > 500
    assert np.array_equal(h[clear], rid[clear])
    np.testing.assert_allclose(t[clear], rt[clear], rtol=1e-5)
    # clearly missed rays miss
    far_miss = ~hit
    assert (h[far_miss] == -1).mean() > 0.99


def test_watertight_closed_mesh(orc):
    """Rays from inside a closed mesh aimed exactly at its vertices and edge
    midpoints must hit something (no cracks), from every origin."""
    tris, _ = synth.uv_spheres(np.array([[0.3, -0.2, 0.1]]), np.array([1.7]), slices=12, bands=11)
    cube = synth.boxes(np.array([[-4.0, -3.0, -5.0]]), np.array([4.5, 3.5, 4.0])[None])
    for mesh in (tris, cube):
        sc = orc.OracleScene(synth.Scene(mesh, np.ones((mesh.shape[0], 3), np.float32)))
        tv = mesh.reshape(-1, 3, 3)
        targets = np.concatenate([tv.reshape(-1, 3), 0.5 * (tv[:, 0] + tv[:, 1]), 0.5 * (tv[:, 1] + tv[:, 2]),
                                  0.5 * (tv[:, 2] + tv[:, 0])]).astype(np.float32)
        for origin in ((0.3, -0.2, 0.1), (0.1, 0.05, -0.3), (-0.2, 0.3, 0.25)):
            o = np.tile(np.array(origin, np.float32), (targets.shape[0], 1))
            dd = (targets - o).astype(np.float64)
            dd /= np.linalg.norm(dd, axis=1, keepdims=True)
            h, _ = orc.closest_hit(sc, o, dd.astype(np.float32))
            assert (h >= 0).all()


def test_two_sided_and_positive_t(orc):
    tri = np.array([[-1, -1, 5, 1, -1, 5, 0, 1, 5]], np.float32)
    sc = orc.OracleScene(synth.Scene(tri, np.ones((1, 3), np.float32)))
    o = np.array([[0, 0, 0], [0, 0, 10], [0, 0, 6]], np.float32)
    d = np.array([[0, 0, 1], [0, 0, -1], [0, 0, 1]], np.float32)
    h, t = orc.closest_hit(sc, o, d)
    assert h.tolist() == [0, 0, -1]
    assert t[0] == 5.0 and t[1] == 5.0


def test_equal_distance_tie_takes_smaller_id(orc):
    # the same triangle twice: equal t, the smaller original id wins
    tri = np.array([[-1, -1, 5, 1, -1, 5, 0, 1, 5]] * 3, np.float32)
    tri[0] += np.float32(10.0)  # move id 0 away
    sc = orc.OracleScene(synth.Scene(tri, np.ones((3, 3), np.float32)))
    h, t = orc.closest_hit(sc, np.zeros((1, 3), np.float32), np.array([[0, 0, 1]], np.float32))
    assert h[0] == 1
    hb, _ = orc.closest_hit(sc, np.zeros((1, 3), np.float32), np.array([[0, 0, 1]], np.float32),
                            use_bvh=False)
    assert hb[0] == 1


def test_gbuffer_plane_depth_and_shading(orc):
    """A fronto-parallel plane at depth Z0: view depth Z0 everywhere, normal
    facing the camera, Lambert colour albedo * (E * n.l + ambient)."""
    z0 = 7.0
    plane = synth.quad((-100, -100, z0), (-100, 100, z0), (100, 100, z0), (100, -100, z0))
    alb = np.array([[0.8, 0.5, 0.25]] * 2, np.float32)
    ldir = synth.f32tuple(synth._normalize((0.3, -0.2, 1.0)))
    sc = orc.OracleScene(synth.Scene(plane, alb, light_dir=ldir))
    cam = synth.look_camera((0, 0, 0), 0.0, 0.0, 32, 24)
    g = orc.gbuffer(sc, cam, synth.Lens())
    np.testing.assert_allclose(g.depth, z0, rtol=2e-6)
    np.testing.assert_allclose(g.normal[..., :3], np.broadcast_to([0, 0, -1], (24, 32, 3)), atol=1e-6)
    ndl = -float(np.dot([0, 0, -1], ldir))
    want = alb[0] * (1.0 * ndl + 0.15)
    np.testing.assert_allclose(g.colour[..., :3], np.broadcast_to(want, (24, 32, 3)), rtol=1e-6)
