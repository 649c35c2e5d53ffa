"""GPU parity: libdof (through its C ABI) against the CPU oracle on the same
seeded inputs, stage by stage, on the 256x256 workload (866 triangles, 4 rays
per masked pixel).  Index work is compared bit for bit; intermediate floats
to 1e-5; the final colour to 1e-3 per linear-RGB channel."""

import dataclasses
import math

import numpy as np
import pytest

from paper_2210_06158_amd import synth

pytestmark = pytest.mark.gpu

LEAF = 0x80000000
COLOUR_TOL = 1e-3
STAGE_TOL = 1e-5


@pytest.fixture(scope="module")
def env(orc):
    import torch
    from paper_2210_06158_amd import dof
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    scene, cam, lens, params = synth.scene_small()
    osc = orc.OracleScene(scene)
    osc.build_bvh()
    gs = dof.Scene(scene)
    gs.build_bvh()
    torch.cuda.synchronize()
    return dict(torch=torch, dof=dof, scene=scene, cam=cam, lens=lens, params=params, osc=osc, gs=gs)


def to_gpu(torch, gb):
    return (torch.from_numpy(gb.colour).cuda(), torch.from_numpy(gb.depth).cuda(), torch.from_numpy(gb.normal).cuda())


def run_pair(env, orc, cam, lens, params, gb, hist_in=None, prev_cam=None, prev_lens=None, fmt16=False, knobs=None):
    torch, dof = env["torch"], env["dof"]
    o = orc.render_frame(env["osc"], cam, lens, params, gb, hist_in=hist_in, prev_cam=prev_cam, prev_lens=prev_lens)
    fr = dof.Frame(cam.width, cam.height, params, ray_records=True, knobs=knobs)
    g = to_gpu(torch, gb)
    if fmt16:
        g = (g[0].half(), g[1], g[2].half())
    hin = torch.from_numpy(hist_in).cuda() if hist_in is not None else None
    hout = dof.history_alloc(cam.width, cam.height)
    fr.render(env["gs"], cam, lens, g, hin, hout, prev_cam=prev_cam, prev_lens=prev_lens)
    torch.cuda.synchronize()
    d = fr.debug()
    d["colour"] = fr.colour.float().cpu().numpy()
    d["mask"] = fr.mask.cpu().numpy()
    d["hist_out"] = hout.cpu().numpy()
    d["stats"] = fr.stats.cpu().numpy()
    return o, d


def compare_frame(o, d, label):
    m = o["mask"] > 0
    assert np.array_equal(d["colr"], o["colr"]), label
    assert np.array_equal(d["zn"], o["zn"]), label
    assert np.array_equal(d["tile_max"], o["tile_max"]) and np.array_equal(d["tile_dil"], o["tile_dil"]), label
    np.testing.assert_allclose(d["pre"], o["pre"], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    np.testing.assert_allclose(d["gather"], o["gather"], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    np.testing.assert_allclose(d["ppmed"], o["ppmed"], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    assert np.array_equal(d["prev_idx"], o["prev_idx"]), label
    assert np.array_equal(d["mask"], o["mask"]), label
    assert d["n_masked"] == o["n_masked"] and d["n_rays"] == o["n_rays"], label
    assert int(d["stats"][0]) == o["n_masked"] and int(d["stats"][1]) == o["n_rays"], label
    assert np.array_equal(d["queue"], o["queue"]) and np.array_equal(d["ray_base"], o["ray_base"]), label
    assert np.array_equal(d["ray_hit"], o["ray_hit"]), label
    assert np.array_equal(d["ray_t"].view(np.uint32), o["ray_t"].view(np.uint32)), label
    np.testing.assert_allclose(d["ray_col"], o["ray_col"], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    np.testing.assert_allclose(d["ray_pos"], o["ray_pos"], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    np.testing.assert_allclose(d["resolve"][:, m], o["resolve"][:, m], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    np.testing.assert_allclose(d["temporal"], o["temporal"], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    np.testing.assert_allclose(d["var_blur"], o["var_blur"], rtol=STAGE_TOL, atol=1e-9, err_msg=label)
    np.testing.assert_allclose(d["rtmed"], o["rtmed"], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    np.testing.assert_allclose(d["mips"], o["mips"], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    np.testing.assert_allclose(d["recon"], o["recon"], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    np.testing.assert_allclose(d["hist_out"], o["hist_out"], rtol=STAGE_TOL, atol=STAGE_TOL, err_msg=label)
    err = np.abs(d["colour"][..., :3] - o["colour"][..., :3]).max()
    assert err <= COLOUR_TOL, (label, err)


# ---------------------------------------------------------------- BVH

def test_bvh_bit_exact(env, orc):
    torch = env["torch"]
    v = env["gs"].bvh_view()
    ob = env["osc"].bvh
    n = v["nleaf"]
    assert n == ob["refs"].size
    keys = v["keys"].cpu().numpy().view(np.uint64)
    refs = v["ids"].cpu().numpy().view(np.uint32)
    assert np.array_equal(keys, ob["keys"])
    assert np.array_equal(refs, ob["refs"])
    nodes = v["nodes"].cpu().numpy().reshape(n - 1, 16)
    nu = nodes.view(np.uint32)
    assert np.array_equal(nu[:, 12], ob["left"][:n - 1]) and np.array_equal(nu[:, 13], ob["right"][:n - 1])
    # leaf ranges: the leaves below each node, from the oracle's child arrays (children's ranges, leftmost
    # and rightmost), and the Karras property that a node's index is an end of its range
    first, last = np.zeros(n - 1, np.int64), np.zeros(n - 1, np.int64)
    def span(c):
        return (c & ~LEAF, c & ~LEAF) if c & LEAF else (first[c], last[c])
    done = np.zeros(n - 1, bool)
    stack = [0]
    while stack:                       # post-order over the oracle's tree
        i = stack[-1]
        kids = [int(ob["left"][i]), int(ob["right"][i])]
        todo = [k for k in kids if not (k & LEAF) and not done[k]]
        if todo:
            stack.extend(todo)
            continue
        stack.pop()
        first[i], last[i] = span(kids[0])[0], span(kids[1])[1]
        done[i] = True
    assert np.array_equal(nu[:, 14], first) and np.array_equal(nu[:, 15], last)
    idx = np.arange(n - 1)
    assert np.all((idx == first) | (idx == last))
    assert np.array_equal(v["parent"].cpu().numpy().view(np.uint32), ob["parent"])

    def child_box(c):
        return ob["leaf_bounds"][c & ~LEAF] if c & LEAF else ob["bounds"][c]
    for i in range(n - 1):
        a, b, c = nodes[i, 0:4], nodes[i, 4:8], nodes[i, 8:12]
        lb = np.array([a[0], a[2], c[0], a[1], a[3], c[1]], np.float32)
        rb = np.array([b[0], b[2], c[2], b[1], b[3], c[3]], np.float32)
        assert np.array_equal(lb.view(np.uint32), child_box(int(ob["left"][i])).view(np.uint32))
        assert np.array_equal(rb.view(np.uint32), child_box(int(ob["right"][i])).view(np.uint32))
    tris = v["tris"].cpu().numpy().reshape(n, 12)
    want = env["scene"].verts[ob["ids"]]
    assert np.array_equal(tris[:, [0, 1, 2, 4, 5, 6, 8, 9, 10]], want)
    assert np.array_equal(tris[:, 3].view(np.uint32), ob["ids"])


def half_words(box):
    """The traversal's binary16 words of child boxes (n, 6: lo xyz, hi xyz):
    per axis the low plane rounded down in bits 0-15 and the high plane
    rounded up in bits 16-31, a result in the subnormal range moved outward to
    0 or 2^-14 (written from the definition with numpy's binary16)."""
    m = np.float32(2.0 ** -14)

    def conv(x, down):
        x = np.asarray(x, np.float32)
        with np.errstate(over="ignore"):
            h = x.astype(np.float16)
        if down:
            h = np.where(h.astype(np.float32) > x, np.nextafter(h, np.float16(-np.inf)), h)
        else:
            h = np.where(h.astype(np.float32) < x, np.nextafter(h, np.float16(np.inf)), h)
        v = h.astype(np.float32)
        sub_pos, sub_neg = (v > 0) & (v < m), (v < 0) & (v > -m)
        v = np.where(sub_pos, np.float32(0) if down else m, np.where(sub_neg, -m if down else np.float32(0), v))
        return v.astype(np.float16).view(np.uint16).astype(np.uint32)

    return np.stack([conv(box[:, a], True) | (conv(box[:, a + 3], False) << 16) for a in range(3)], 1)


def check_nodes16(view, lbox, rbox, left, right):
    """The binary16 node copy: both children's boxes rounded outward and the
    child links, word for word."""
    nl = view["nleaf"]
    got = view["nodes16"].cpu().numpy().view(np.uint32).reshape(nl - 1, 8)
    want = np.concatenate([half_words(lbox), half_words(rbox)], 1)
    assert np.array_equal(got[:, :6], want)
    assert np.array_equal(got[:, 6], left[:nl - 1]) and np.array_equal(got[:, 7], right[:nl - 1])


@pytest.mark.parametrize("n,seed,split", [(1, 3, 2), (2, 4, 2), (3, 5, 2), (257, 6, 2), (5000, 7, 2), (5000, 8, 1),
                                          (5000, 9, 3), (2000, 10, 0)])
def test_bvh_random_soups_and_closest_hit(env, orc, n, seed, split):
    """Random soups (many thin triangles) with each leaf split: keys, leaf
    references, children, child boxes and leaf triangles bit for bit, and
    every ray's closest hit equal to brute force over the triangles."""
    torch, dof = env["torch"], env["dof"]
    v, a = synth.random_triangles(n, seed=seed, spread=4.0, size=0.8)
    sc = synth.Scene(v, a, leaf_split=split)
    osc = orc.OracleScene(sc)
    ob = osc.build_bvh()
    gs = dof.Scene(sc)
    gs.build_bvh()
    torch.cuda.synchronize()
    view = gs.bvh_view()
    nl = view["nleaf"]
    assert nl == ob["refs"].size and (n < 100 or (nl > n) == (split > 0))   # the larger soups have thin triangles
    keys = view["keys"].cpu().numpy().view(np.uint64)
    refs = view["ids"].cpu().numpy().view(np.uint32)
    assert np.array_equal(keys, ob["keys"]) and np.array_equal(refs, ob["refs"])
    if nl > 1:
        nodes = view["nodes"].cpu().numpy().reshape(nl - 1, 16)
        nu = nodes.view(np.uint32)
        assert np.array_equal(nu[:, 12], ob["left"][:nl - 1]) and np.array_equal(nu[:, 13], ob["right"][:nl - 1])
        # child boxes bit for bit: split references carry clipped boxes
        lb = np.stack([nodes[:, 0], nodes[:, 2], nodes[:, 8], nodes[:, 1], nodes[:, 3], nodes[:, 9]], 1)
        rb = np.stack([nodes[:, 4], nodes[:, 6], nodes[:, 10], nodes[:, 5], nodes[:, 7], nodes[:, 11]], 1)
        def boxes_of(ch):
            ch = ch[:nl - 1].astype(np.int64)
            leaf = (ch & 0x80000000) != 0
            out = np.where(leaf[:, None], ob["leaf_bounds"][np.where(leaf, ch & 0x7FFFFFFF, 0)],
                           ob["bounds"][np.where(leaf, 0, ch)])
            return out.astype(np.float32)
        assert np.array_equal(lb.view(np.uint32), boxes_of(ob["left"]).view(np.uint32))
        assert np.array_equal(rb.view(np.uint32), boxes_of(ob["right"]).view(np.uint32))
        check_nodes16(view, boxes_of(ob["left"]), boxes_of(ob["right"]), ob["left"], ob["right"])
    tris = view["tris"].cpu().numpy().reshape(nl, 12)
    assert np.array_equal(tris[:, 3].view(np.uint32), ob["ids"])
    assert np.array_equal(tris[:, [0, 1, 2, 4, 5, 6, 8, 9, 10]], v[ob["ids"]])
    rng = synth.SplitMix64(seed * 31)
    nr = 20000
    o = rng.uniform(3 * nr, -5, 5).reshape(nr, 3).astype(np.float32)
    t = rng.uniform(3 * nr, -3, 3).reshape(nr, 3)
    d = (t - o).astype(np.float32)
    hg, tg = gs.trace_rays(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda())
    ho, to = orc.closest_hit(osc, o, d, use_bvh=False)
    assert np.array_equal(hg.cpu().numpy(), ho)
    assert np.array_equal(tg.cpu().numpy().view(np.uint32), to.view(np.uint32))



def test_rays_lying_on_a_box_face(env, orc):
    """Rays parallel to an axis (a direction component of exactly 0) that lie
    in a face of a leaf's box and cross the triangle's edge in that face: the
    watertight test counts the edge hit, so the box test must not cull the
    leaf.  Faces at the high and the low end of z and x.  GPU, oracle BVH and
    oracle brute force agree on every id and distance."""
    torch, dof = env["torch"], env["dof"]
    tri = np.array([
        [0, 0, 2, 2, 0, 2, 1, 0, 1],        # edge in z = 2, the top face of its box
        [5, 5, 5, 6, 5, 5, 5, 6, 6],        # elsewhere, so the root box is larger than the leaves
        [4, 0, 1, 6, 0, 1, 5, 0, 2],        # edge in z = 1, the bottom face
        [8, 0, 0, 8, 0, 1, 7, 0, 0.5],      # edge in x = 8, the high x face
        [10, 0, 0, 10, 0, 1, 11, 0, 0.5],   # edge in x = 10, the low x face
    ], np.float32)
    sc = synth.Scene(tri, np.full((len(tri), 3), 0.5, np.float32))
    osc = orc.OracleScene(sc)
    osc.build_bvh()
    gs = dof.Scene(sc)
    gs.build_bvh()
    o = np.array([[1, -1, 2], [1, 1, 2], [0.5, -3, 2], [5, -1, 1], [8, -1, 0.5], [8, 2, 0.5], [10, -1, 0.5]],
                 np.float32)
    d = np.array([[0, 1, 0], [0, -1, 0], [0, 1, 0], [0, 1, 0], [0, 1, 0], [0, -1, 0], [0, 1, 0]], np.float32)
    hb, tb = orc.closest_hit(osc, o, d, use_bvh=True)
    ho, to = orc.closest_hit(osc, o, d, use_bvh=False)
    assert np.array_equal(ho, [0, 0, 0, 2, 3, 3, 4]) and np.array_equal(to, [1, 1, 3, 1, 1, 2, 1])
    assert np.array_equal(hb, ho) and np.array_equal(tb, to)
    hg, tg = gs.trace_rays(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda())
    assert np.array_equal(hg.cpu().numpy(), ho)
    assert np.array_equal(tg.cpu().numpy().view(np.uint32), to.view(np.uint32))


def morton_cell(code):
    """Integer cell (x, y, z) of a 63-bit Morton code (bit 3i+2 is x, 3i+1 y,
    3i z)."""
    x = y = z = 0
    for i in range(21):
        z |= ((code >> (3 * i)) & 1) << i
        y |= ((code >> (3 * i + 1)) & 1) << i
        x |= ((code >> (3 * i + 2)) & 1) << i
    return float(x), float(y), float(z)


def ladder_scene():
    """A tree about 62 levels deep in which every level has two internal
    children: triangle centroids on the Morton codes 0, 1 and 2^k, 2^k + 1
    (k = 1..62), plus one at (2^21, 2^21, 2^21) that fixes the grid to unit
    cells.  The top split at level k separates the pair {2^k, 2^k + 1} (an
    internal node with two leaves) from the rest.  Every triangle is huge
    and they all overlap, so a ray enters both children everywhere; the
    remaining chain's box contains the pair's, so the chain is the near child
    and the pair is pushed, about 62 entries: the LDS stack (16, 24 or 32
    entries) overflows, its oldest entries are dropped and must be found
    again by walking parent links.  The three vertex depths are permuted per
    triangle (bounds and centroid unchanged), so the planes tilt differently
    and the closest hit varies across rays; a traversal that lost the dropped
    entries returns a different hit for many of them."""
    import itertools
    S = float(2 ** 23)
    codes = [0, 1]
    for k in range(1, 63):
        codes += [1 << k, (1 << k) + 1]
    cents = [morton_cell(c) for c in codes] + [(2.0 ** 21, 2.0 ** 21, 2.0 ** 21)]
    perms = list(itertools.permutations((-1.0, 1.0, 0.0)))
    tris = []
    for i, (cx, cy, cz) in enumerate(cents):
        p = perms[(i * 7 + i // 5) % 6]
        tris.append([cx - S, cy - S, cz + p[0] * S, cx + S, cy - S, cz + p[1] * S, cx, cy + S, cz + p[2] * S])
    v = np.array(tris, np.float32)
    return synth.Scene(v, np.ones((v.shape[0], 3), np.float32))


def ladder_rungs(ob, n):
    """Internal nodes of the oracle's tree whose two children are internal."""
    left, right = ob["left"][:n - 1], ob["right"][:n - 1]
    return int(np.sum(((left & LEAF) == 0) & ((right & LEAF) == 0)))


@pytest.fixture(scope="module")
def ladder(env, orc):
    dof = env["dof"]
    sc = ladder_scene()
    osc = orc.OracleScene(sc)
    ob = osc.build_bvh()
    gs = dof.Scene(sc)
    gs.build_bvh()
    env["torch"].cuda.synchronize()
    assert ladder_rungs(ob, sc.ntri) >= 60
    return sc, osc, ob, gs


def test_deep_tree_stack_drops(env, orc, ladder):
    torch = env["torch"]
    sc, osc, ob, gs = ladder
    view = gs.bvh_view()
    assert np.array_equal(view["keys"].cpu().numpy().view(np.uint64), ob["keys"])
    n = view["nleaf"]
    nu = view["nodes"].cpu().numpy().reshape(n - 1, 16).view(np.uint32)
    assert np.array_equal(nu[:, 12], ob["left"][:n - 1]) and np.array_equal(nu[:, 13], ob["right"][:n - 1])
    rng = synth.SplitMix64(99)
    nr = 4096
    o = np.stack([rng.uniform(nr, -2e6, 2e6), rng.uniform(nr, -2e6, 2e6), np.full(nr, -3e7)], 1).astype(np.float32)
    d = np.stack([rng.uniform(nr, -0.1, 0.1), rng.uniform(nr, -0.1, 0.05), np.ones(nr)], 1).astype(np.float32)
    hg, tg = gs.trace_rays(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda())
    ho, to = orc.closest_hit(osc, o, d, use_bvh=False)
    assert (ho >= 0).mean() > 0.9 and np.unique(ho).size >= 8
    assert np.array_equal(hg.cpu().numpy(), ho)
    assert np.array_equal(tg.cpu().numpy().view(np.uint32), to.view(np.uint32))


@pytest.mark.parametrize("stack", [16, 24, 32])
def test_deep_tree_frame_with_each_stack_depth(env, orc, ladder, stack):
    """The frame pass's lens rays on the ladder tree with each LDS stack
    depth: the frame counts its drops, and every ray's hit and distance equal
    the oracle's (whose traversal recurses without a depth limit)."""
    sc, osc, _, gs = ladder
    cam = synth.Camera(pos=(0.0, 0.0, -3.0e7), right=(1.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), fwd=(0.0, 0.0, 1.0),
                       width=64, height=48)
    lens = synth.Lens(focal=0.1, fnum=1.4, focus=3.0e7)
    params = synth.Params(m=4, mask_mode=synth.MASK_ALL)
    gb = orc.gbuffer(osc, cam, lens)
    o, d = run_pair(dict(env, osc=osc, gs=gs), orc, cam, lens, params, gb, knobs={"trace_stack": stack})
    assert o["n_rays"] == 32 * 24 * 4 and int(d["stats"][1]) == o["n_rays"]
    assert int(d["stats"][6]) > 0, "no stack drops: the test does not reach the parent walk"
    assert np.unique(o["ray_hit"]).size >= 8
    assert np.array_equal(d["ray_hit"], o["ray_hit"])
    assert np.array_equal(d["ray_t"].view(np.uint32), o["ray_t"].view(np.uint32))


def test_watertight_on_gpu(env, orc):
    torch, dof = env["torch"], env["dof"]
    mesh, _ = synth.uv_spheres(np.array([[0.3, -0.2, 0.1]]), np.array([1.7]))
    sc = synth.Scene(mesh, np.ones((mesh.shape[0], 3), np.float32))
    gs = dof.Scene(sc)
    gs.build_bvh()
    tv = mesh.reshape(-1, 3, 3)
    targets = np.concatenate([tv.reshape(-1, 3), 0.5 * (tv[:, 0] + tv[:, 1])]).astype(np.float32)
    o = np.tile(np.array([0.3, -0.2, 0.1], np.float32), (targets.shape[0], 1))
    hg, _ = gs.trace_rays(torch.from_numpy(o).cuda(), torch.from_numpy(targets - o).cuda())
    assert (hg.cpu().numpy() >= 0).all()


# ---------------------------------------------------------------- G-buffer

@pytest.mark.parametrize("jitter", [(0.0, 0.0), (0.37, -0.21)])
def test_gbuffer_matches_oracle(env, orc, jitter):
    torch = env["torch"]
    cam = dataclasses.replace(env["cam"], jitter=jitter)
    og = orc.gbuffer(env["osc"], cam, env["lens"])
    c, dpt, nrm = env["gs"].render_gbuffer(cam, env["lens"])
    torch.cuda.synchronize()
    assert np.array_equal(dpt.cpu().numpy().view(np.uint32), og.depth.view(np.uint32))
    assert np.array_equal(c.cpu().numpy(), og.colour)
    assert np.array_equal(nrm.cpu().numpy(), og.normal)


# ---------------------------------------------------------------- frames

@pytest.fixture(scope="module")
def frame0(env, orc):
    gb = orc.gbuffer(env["osc"], env["cam"], env["lens"])
    o, d = run_pair(env, orc, env["cam"], env["lens"], env["params"], gb)
    return gb, o, d


def test_frame0_parity(frame0):
    _, o, d = frame0
    compare_frame(o, d, "frame 0")
    assert o["n_rays"] > 1000


def test_frame1_pan_parity(env, orc, frame0):
    """Second frame after a 0.02-unit pan, both sides fed the oracle's
    history of frame 0 (motion: reduced blend, latest hit ratio)."""
    _, o0, _ = frame0
    cam1 = synth.pan_camera(env["cam"], 0.02)
    gb1 = orc.gbuffer(env["osc"], cam1, env["lens"])
    o, d = run_pair(env, orc, cam1, env["lens"], env["params"], gb1, hist_in=o0["hist_out"],
                    prev_cam=env["cam"], prev_lens=env["lens"])
    assert (o["prev_idx"] >= 0).mean() > 0.5
    compare_frame(o, d, "frame 1 pan")


def test_frame1_static_parity(env, orc, frame0):
    gb, o0, _ = frame0
    cam1 = dataclasses.replace(env["cam"], frame=1)
    o, d = run_pair(env, orc, cam1, env["lens"], env["params"], gb, hist_in=o0["hist_out"],
                    prev_cam=env["cam"], prev_lens=env["lens"])
    compare_frame(o, d, "frame 1 static")


def test_fp16_gbuffer_parity(env, orc):
    """FP16 colour/normal G-buffer: the oracle reads the same values widened
    to binary32 (exact), so parity holds at the same tolerances."""
    gb = orc.gbuffer(env["osc"], env["cam"], env["lens"])
    gb16 = orc.GBuffer(gb.colour.astype(np.float16).astype(np.float32), gb.depth,
                       gb.normal.astype(np.float16).astype(np.float32))
    o, d = run_pair(env, orc, env["cam"], env["lens"], env["params"], gb16, fmt16=True)
    compare_frame(o, d, "fp16 G-buffer")


@pytest.mark.parametrize("mode,m", [(synth.MASK_ALL, 3), (synth.MASK_FIXED, 5), (synth.MASK_DILATE, 4)])
def test_mask_modes_parity(env, orc, frame0, mode, m):
    gb, _, _ = frame0
    p = dataclasses.replace(env["params"], mask_mode=mode, m=m)
    o, d = run_pair(env, orc, env["cam"], env["lens"], p, gb)
    compare_frame(o, d, f"mask mode {mode}")


def test_literal_composite_reading_parity(env, orc, frame0):
    """The far-field blend read literally (composite_literal = 1): the whole
    frame against the oracle, and the output differs from the default
    reading's where far-field pixels blend."""
    gb, _, d0 = frame0
    p = dataclasses.replace(env["params"], composite_literal=1)
    o, d = run_pair(env, orc, env["cam"], env["lens"], p, gb)
    compare_frame(o, d, "literal composite")
    assert np.abs(d["colour"] - d0["colour"]).max() > 1e-3


def test_gather_windows_parity(env, orc, frame0):
    """The gather with every LDS window the tuner may pick (and none): the
    prefiltered/gathered planes against the oracle, and identical to each
    other bit for bit (one tap arithmetic in both variants)."""
    gb, _, d0 = frame0
    for win in (-1, 32, 40):
        o, d = run_pair(env, orc, env["cam"], env["lens"], env["params"], gb, knobs={"gather_window": win})
        compare_frame(o, d, f"gather window {win}")
        assert np.array_equal(d["gather"], d0["gather"]), win


def test_reconstruction_global_fallback_parity(env, orc):
    """Blocks whose mip footprint does not fit the reconstruction's LDS
    staging buffer read the mips in global memory.  A wide aperture (bar
    CoCs near 70 px) with lod_scale 0.01 keeps tap radii of 12+ half-res px on
    mip level 0, so such blocks need more than 2,700 texels, beyond the 2,496
    staged; other blocks of the same frames stay staged.  Two frames, the
    second on the first's history, with a variance weight that puts the
    blend factor b at its cap, so the taps decide the result."""
    lens = dataclasses.replace(env["lens"], focal=0.15, fnum=1.0)
    p = dataclasses.replace(env["params"], lod_scale=0.01, mask_mode=synth.MASK_ALL, var_recon_w=1e6)
    gb = orc.gbuffer(env["osc"], env["cam"], lens)
    o0, d0 = run_pair(env, orc, env["cam"], lens, p, gb)
    compare_frame(o0, d0, "recon fallback, frame 0")
    cam1 = dataclasses.replace(env["cam"], frame=1)
    o1, d1 = run_pair(env, orc, cam1, lens, p, gb, hist_in=o0["hist_out"], prev_cam=env["cam"], prev_lens=lens)
    ct = o1["temporal"][1][..., 0]
    traced = o1["temporal"][0][..., 3] > 0
    big = traced & (ct * p.lod_scale < 1.0) & (ct * 0.25 >= 12.0)
    assert big.sum() > 50                                               # level-0 radii that overflow a block
    bb = np.clip(o1["var_blur"] * p.var_recon_w, 0.0, p.b_max)
    assert (bb[big] > 0.5).mean() > 0.9                                 # the taps decide the result there
    compare_frame(o1, d1, "recon fallback, frame 1")


@pytest.mark.parametrize("lod_scale,lod_max", [(0.2, 1.0), (0.05, 0.0)])
def test_reconstruction_mip_level_limits_parity(env, orc, lod_scale, lod_max):
    """Eq. (8) with a lower top level: lod_max 1 puts most pixels on levels 1
    and 1 (both samples from one level, whose staged box then serves both),
    lod_max 0 leaves only the finest level.  Second frame on the first's
    history, blend factor b at its cap, so the taps decide the result."""
    lens = dataclasses.replace(env["lens"], focal=0.15, fnum=1.0)
    p = dataclasses.replace(env["params"], lod_scale=lod_scale, lod_max=lod_max, mask_mode=synth.MASK_ALL,
                            var_recon_w=1e6)
    gb = orc.gbuffer(env["osc"], env["cam"], lens)
    o0, d0 = run_pair(env, orc, env["cam"], lens, p, gb)
    compare_frame(o0, d0, f"lod_max {lod_max}, frame 0")
    cam1 = dataclasses.replace(env["cam"], frame=1)
    o1, d1 = run_pair(env, orc, cam1, lens, p, gb, hist_in=o0["hist_out"], prev_cam=env["cam"], prev_lens=lens)
    ct = o1["temporal"][1][..., 0]
    traced = o1["temporal"][0][..., 3] > 0
    lod = np.clip(ct * lod_scale, 0.0, lod_max)
    assert (lod[traced] >= lod_max).mean() > 0.2                       # many pixels at the top level
    compare_frame(o1, d1, f"lod_max {lod_max}, frame 1")

@pytest.mark.parametrize("polygon", [0, 1])
def test_hexagon_aperture_and_ragged_size(env, orc, polygon):
    """6-blade aperture at a size that is not a multiple of any tile
    (ragged tails in every kernel); with polygon = 1 the post-process gather
    samples the hexagon too."""
    lens = dataclasses.replace(env["lens"], fnum=2.0, blades=6, blade_rot=0.2)
    cam = dataclasses.replace(env["cam"], width=202, height=118)
    gb = orc.gbuffer(env["osc"], cam, lens)
    o, d = run_pair(env, orc, cam, lens, dataclasses.replace(env["params"], m=6, pp_polygon=polygon), gb)
    compare_frame(o, d, f"hexagon 202x118 polygon={polygon}")


def test_pinhole_reduction_on_gpu(env, orc):
    lens = dataclasses.replace(env["lens"], fnum=math.inf)
    gb = orc.gbuffer(env["osc"], env["cam"], lens)
    o, d = run_pair(env, orc, env["cam"], lens, env["params"], gb)
    assert np.array_equal(d["colour"][..., :3].view(np.uint32), gb.colour[..., :3].view(np.uint32))


def test_determinism_run_twice(env, orc, frame0):
    gb, _, d0 = frame0
    _, d1 = run_pair(env, orc, env["cam"], env["lens"], env["params"], gb)
    for k in ("colour", "mask", "queue", "ray_hit", "ray_col", "recon", "hist_out"):
        assert np.array_equal(d0[k], d1[k]), k


# ---------------------------------------------------------------- final TAA

@pytest.fixture(scope="module")
def taa0(env, orc, frame0):
    gb, _, _ = frame0
    p = dataclasses.replace(env["params"], taa=1)
    o, d = run_pair(env, orc, env["cam"], env["lens"], p, gb)
    return p, o, d


def test_taa_frame0_is_the_composite(taa0, frame0):
    """Without history the final TAA passes the composite through: same
    stages and colour as the frame without TAA, and the TAA history plane
    holds that colour."""
    _, o, d = taa0
    _, o_plain, d_plain = frame0
    compare_frame(o, d, "TAA frame 0")
    assert np.array_equal(d["colour"][..., :3], d_plain["colour"][..., :3])
    W, H = o["colour"].shape[1], o["colour"].shape[0]
    from oracle import taa_offset
    plane = d["hist_out"][taa_offset(W, H):taa_offset(W, H) + 4 * W * H].reshape(H, W, 4)
    assert np.array_equal(plane[..., :3], d["colour"][..., :3])


def test_taa_frame1_pan_parity(env, orc, taa0):
    """Second frame after a pan, both sides fed the oracle's TAA history of
    frame 0: reprojected, clamped history blended at weight 0.9."""
    p, o0, _ = taa0
    cam1 = synth.pan_camera(env["cam"], 0.02)
    gb1 = orc.gbuffer(env["osc"], cam1, env["lens"])
    o, d = run_pair(env, orc, cam1, env["lens"], p, gb1, hist_in=o0["hist_out"], prev_cam=env["cam"],
                    prev_lens=env["lens"])
    compare_frame(o, d, "TAA frame 1 pan")
    plain = orc.render_frame(env["osc"], cam1, env["lens"], dataclasses.replace(p, taa=0), gb1,
                             hist_in=o0["hist_out"], prev_cam=env["cam"], prev_lens=env["lens"])
    assert np.abs(plain["colour"][..., :3] - o["colour"][..., :3]).max() > 1e-3   # the history took part


def test_taa_all_stages_on_jittered_frames_parity(env, orc):
    """Raster, post-filter and final TAA on a jittered camera path (seeded
    sub-pixel offsets per frame): frame 0, then frame 1 after a pan on the
    oracle's history of frame 0.  Every stage, the history record with its
    three TAA planes and the colour are compared as for plain frames."""
    lens = env["lens"]
    p = dataclasses.replace(env["params"], taa=synth.TAA_ALL)
    cams = synth.jittered([env["cam"], synth.pan_camera(env["cam"], 0.02)], seed=synth.BASE_SEED + 31)
    assert all(c.jitter != (0.0, 0.0) for c in cams)
    gb0 = orc.gbuffer(env["osc"], cams[0], lens)
    o0, d0 = run_pair(env, orc, cams[0], lens, p, gb0)
    compare_frame(o0, d0, "TAA all, jittered frame 0")
    gb1 = orc.gbuffer(env["osc"], cams[1], lens)
    o1, d1 = run_pair(env, orc, cams[1], lens, p, gb1, hist_in=o0["hist_out"], prev_cam=cams[0], prev_lens=lens)
    compare_frame(o1, d1, "TAA all, jittered frame 1")
    plain = orc.render_frame(env["osc"], cams[1], lens, env["params"], gb1, hist_in=o0["hist_out"],
                             prev_cam=cams[0], prev_lens=lens)
    assert not np.array_equal(plain["colr"], o1["colr"])                  # the raster TAA took part


def test_single_frame_graph_replays(env, orc):
    """dof_render_frame captured in a HIP graph -- its post-process chain
    forks to the scene's side stream and joins back before the composite,
    both inside the graph -- and replayed three times with new G-buffer
    contents and eager work in between: every replay equals the eager frame
    of the same inputs (colour, mask, history)."""
    torch, dof = env["torch"], env["dof"]
    cam, lens, params = env["cam"], env["lens"], env["params"]
    W, H = cam.width, cam.height
    gbs = [orc.gbuffer(env["osc"], synth.pan_camera(cam, 0.01 * k) if k else cam, lens) for k in range(3)]
    g_in = to_gpu(torch, gbs[0])
    fr = dof.Frame(W, H, params)
    hout = dof.history_alloc(W, H)
    fr.render(env["gs"], cam, lens, g_in, None, hout)            # warm-up outside the capture
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            fr.render(env["gs"], cam, lens, g_in, None, hout)
    torch.cuda.synchronize()
    for rep, gb in enumerate(reversed(gbs)):
        src = to_gpu(torch, gb)
        ref, ref_h = dof.Frame(W, H, params), dof.history_alloc(W, H)
        ref.render(env["gs"], cam, lens, src, None, ref_h)
        for dst, s in zip(g_in, src):
            dst.copy_(s)
        junk = torch.randn(1 << 20, device="cuda").sum()           # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(fr.colour, ref.colour), rep
        assert torch.equal(fr.mask, ref.mask) and torch.equal(hout, ref_h), rep


@pytest.mark.parametrize("split", [1, 2, 3])
def test_leaf_split_edge_cases(env, orc, split):
    """Reference boxes, keys and tree bit for bit and every closest hit equal
    to brute force on the awkward soup, at each split level."""
    torch, dof = env["torch"], env["dof"]
    v, a, o, d = synth.awkward_triangles(4242)
    sc = synth.Scene(v, a, leaf_split=split)
    osc = orc.OracleScene(sc)
    ob = osc.build_bvh()
    gs = dof.Scene(sc)
    gs.build_bvh()
    torch.cuda.synchronize()
    view = gs.bvh_view()
    nl = view["nleaf"]
    assert nl == ob["refs"].size and nl > v.shape[0]
    assert np.array_equal(view["keys"].cpu().numpy().view(np.uint64), ob["keys"])
    assert np.array_equal(view["ids"].cpu().numpy().view(np.uint32), ob["refs"])
    nodes = view["nodes"].cpu().numpy().reshape(nl - 1, 16)
    nu = nodes.view(np.uint32)
    assert np.array_equal(nu[:, 12], ob["left"][:nl - 1]) and np.array_equal(nu[:, 13], ob["right"][:nl - 1])
    lb = np.stack([nodes[:, 0], nodes[:, 2], nodes[:, 8], nodes[:, 1], nodes[:, 3], nodes[:, 9]], 1)
    rb = np.stack([nodes[:, 4], nodes[:, 6], nodes[:, 10], nodes[:, 5], nodes[:, 7], nodes[:, 11]], 1)
    want_boxes = []
    for ch, got in ((ob["left"], lb), (ob["right"], rb)):
        ch = ch[:nl - 1].astype(np.int64)
        leaf = (ch & 0x80000000) != 0
        want = np.where(leaf[:, None], ob["leaf_bounds"][np.where(leaf, ch & 0x7FFFFFFF, 0)],
                        ob["bounds"][np.where(leaf, 0, ch)]).astype(np.float32)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
        want_boxes.append(want)
    check_nodes16(view, want_boxes[0], want_boxes[1], ob["left"], ob["right"])
    hg, tg = gs.trace_rays(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda())
    ho, to = orc.closest_hit(osc, o, d, use_bvh=False)
    assert (ho >= 0).mean() > 0.3
    assert np.array_equal(hg.cpu().numpy(), ho)
    assert np.array_equal(tg.cpu().numpy().view(np.uint32), to.view(np.uint32))
