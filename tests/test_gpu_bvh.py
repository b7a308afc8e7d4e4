"""BVH invariants on the device-built tree: every surfel in exactly one
leaf, every child box inside its parent's box, each leaf's box contains its
surfel's k_sigma ellipse, and the stack bound (max depth) is consistent."""
import numpy as np
import pytest
import torch

import scenegen as sg
from tests._util import gpu_scene

pytestmark = pytest.mark.gpu


def _slice(buf, addr, nbytes):
    off = int(addr) - buf.data_ptr()
    assert 0 <= off and off + nbytes <= buf.numel()
    return buf[off:off + nbytes].cpu().numpy()


def _nodes(bvh, n):
    """Copy the node array and permutation out of the BVH's own tensor."""
    info = bvh.info()
    m = max(n - 1, 1)
    nodes = _slice(bvh.mem, info.nodes, m * 64).view(np.int32).reshape(m, 16)
    perm = _slice(bvh.mem, info.perm, n * 4).view(np.int32)
    return info, nodes, perm


def _scene(which):
    return sg.cloud_scene(2000, seed=1) if which == "cloud" else sg.room_scene(30000, (4.0, 3.0, 2.5), 5, seed=8)


def _check_binary(scene, bvh):
    """Binary tree: every surfel in exactly one leaf, every child box inside
    its parent's box, each leaf box around its surfel's centre, and the
    reported depth (levels of internal nodes). Returns the depth."""
    n = scene.n
    info, nodes, perm = _nodes(bvh, n)
    assert sorted(perm.tolist()) == list(range(n))
    boxes = nodes[:, :12].view(np.float32).reshape(-1, 2, 6)       # [node, child, lo3 hi3]
    kids = nodes[:, 12:14]
    seen = np.zeros(n, dtype=np.int64)
    depth_max = 0
    stack = [(0, 0, None)]
    while stack:
        i, d, parent_box = stack.pop()
        depth_max = max(depth_max, d + 1)
        for c in range(2):
            b = boxes[i, c]
            assert np.all(b[:3] <= b[3:])
            if parent_box is not None:
                assert np.all(b[:3] >= parent_box[:3]) and np.all(b[3:] <= parent_box[3:])
            ref = int(kids[i, c])
            if ref >= 0:
                stack.append((ref, d + 1, b))
            else:
                seen[~ref] += 1
                s = int(perm[~ref])
                p = scene.pos[:, s].astype(np.float64)
                assert np.all(b[:3] < p) and np.all(p < b[3:])
    assert np.all(seen == 1)
    assert info.max_depth == depth_max
    lo, hi = np.array(info.lo), np.array(info.hi)
    assert np.all(lo <= scene.pos.min(axis=1)) and np.all(hi >= scene.pos.max(axis=1))
    return depth_max


def _check_wide(scene, bvh):
    """The 4-wide tree the tracer walks: every surfel in exactly one leaf
    slot, every child box inside its parent's box and around its surfel's
    centre, and the reported depth."""
    n = scene.n
    info = bvh.info()
    m = info.n_nodes4
    assert 1 <= m <= n - 1
    raw = _slice(bvh.mem, info.nodes4, m * 128).view(np.int32).reshape(m, 32)
    boxes = raw[:, :24].view(np.float32).reshape(m, 4, 6)
    refs = raw[:, 24:28]
    perm = _slice(bvh.mem, info.perm, n * 4).view(np.int32)
    seen = np.zeros(n, dtype=np.int64)
    visited = np.zeros(m, dtype=np.int64)
    depth = 0
    stack = [(0, 1, None)]
    while stack:
        i, d, pbox = stack.pop()
        visited[i] += 1
        depth = max(depth, d)
        for k in range(4):
            r = int(refs[i, k])
            if r == 0x7FFFFFFF:
                continue
            b = boxes[i, k]
            assert np.all(b[:3] <= b[3:])
            if pbox is not None:
                assert np.all(b[:3] >= pbox[:3]) and np.all(b[3:] <= pbox[3:])
            if r >= 0:
                stack.append((r, d + 1, b))
            else:
                seen[~r] += 1
                p = scene.pos[:, int(perm[~r])].astype(np.float64)
                assert np.all(b[:3] < p) and np.all(p < b[3:])
    assert np.all(seen == 1) and np.all(visited == 1)
    assert info.depth4 == depth
    return depth


@pytest.mark.parametrize("which", ["cloud", "room"])
def test_bvh_invariants(which):
    from paper_2601_23065_amd.api import BVH
    scene = _scene(which)
    bvh = BVH(gpu_scene(scene))
    depth = _check_binary(scene, bvh)
    # the clustering's height bound: 64 iterations plus ceil(log2 n) halvings
    assert depth <= 64 + int(np.ceil(np.log2(scene.n)))


@pytest.mark.parametrize("which", ["cloud", "room"])
def test_bvh4_invariants(which):
    from paper_2601_23065_amd.api import BVH
    scene = _scene(which)
    _check_wide(scene, BVH(gpu_scene(scene)))


def _spread3(x):
    x = x.astype(np.uint64) & np.uint64(0x1FFFFF)
    for shift, mask in ((32, 0x1F00000000FFFF), (16, 0x1F0000FF0000FF), (8, 0x100F00F00F00F00F),
                        (4, 0x10C30C30C30C30C3), (2, 0x1249249249249249)):
        x = (x | (x << np.uint64(shift))) & np.uint64(mask)
    return x


@pytest.mark.parametrize("which", ["cloud", "room"])
def test_sorted_order_is_the_stable_morton_order(which):
    """The leaf order (perm) is the stable sort of the surfels by the 63-bit
    Morton code of their centres on cubic cells of the centres' largest
    extent: integer work, checked bit for bit against the same codes and a
    stable sort computed here (float32 steps as the build takes them)."""
    from paper_2601_23065_amd.api import BVH
    scene = _scene(which)
    n = scene.n
    bvh = BVH(gpu_scene(scene))
    perm = _slice(bvh.mem, bvh.info().perm, n * 4).view(np.int32)
    pos = scene.pos.astype(np.float32)
    lo, hi = pos.min(axis=1), pos.max(axis=1)
    ext = np.float32(max(np.float32(hi[a] - lo[a]) for a in range(3)))
    q = []
    for a in range(3):
        x = np.clip((pos[a] - lo[a]) / ext, np.float32(0.0), np.float32(1.0)).astype(np.float32)
        q.append(np.minimum((x * np.float32(2097152.0)).astype(np.uint32), np.uint32(2097151)))
    code = (_spread3(q[0]) << np.uint64(2)) | (_spread3(q[1]) << np.uint64(1)) | _spread3(q[2])
    want = np.argsort(code, kind="stable")
    assert np.array_equal(perm, want.astype(np.int32))


def test_coincident_surfels_take_the_halving_fallback():
    """600 surfels with one centre, frame and scale: every pair's union has
    the same area, so each clustering iteration merges only the pair at the
    lowest positions (a chain), and the halving iterations finish the tree.
    The trees keep their invariants, the height reaches past 64 levels but
    stays within 64 + ceil(log2 n), and rays through the stack blend the
    surfels in index order as the oracle does, through a hit list that
    overflows."""
    from paper_2601_23065_amd.api import BVH, Params
    from tests.test_gpu_trace import _compare
    n = 600
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)   # noqa: E731
    rng = np.random.default_rng(77)
    rot = np.zeros((4, n))
    rot[0] = 1.0
    scene = sg.Scene(f32(np.zeros((3, n))), f32(rot), f32(np.full((2, n), 0.2)), f32(np.full(n, 0.02)),
                     f32(rng.uniform(0.1, 0.8, (3, n))), f32(rng.uniform(1.0, 10.0, (3, n))), f32(np.ones(n)),
                     bounds=(np.full(3, -1.0), np.full(3, 1.0)))
    bvh = BVH(gpu_scene(scene))
    depth = _check_binary(scene, bvh)
    print(f"binary depth {depth}, 4-wide depth {_check_wide(scene, bvh)}")
    assert 64 < depth <= 64 + int(np.ceil(np.log2(n)))
    m = 64
    O = np.zeros((3, m), dtype=np.float32)
    O[:2] = rng.uniform(-0.2, 0.2, (2, m))
    O[2] = -2.3   # (t = 2.3: away from a depth-bucket edge)
    D = np.zeros((3, m), dtype=np.float32)
    D[2] = 1.0
    segs, _ = _compare(scene, O, D, Params())
    assert min(s.hits.size for s in segs) > 256
    # a refit of this tree (every node made by one clustering or halving
    # iteration) after moving half the surfels matches a fresh build's trace
    from paper_2601_23065_amd.api import trace_rays
    moved = scene.copy()
    moved.pos[0, ::2] += np.float32(0.05)
    gs2 = gpu_scene(moved)
    bvh.refit(gs2)
    _check_binary(moved, bvh)
    fresh = BVH(gs2)
    Ot, Dt = torch.from_numpy(O).cuda(), torch.from_numpy(D).cuda()
    a = trace_rays(bvh, gs2, Params(), Ot, Dt, max_hits=256)
    b = trace_rays(fresh, gs2, Params(), Ot, Dt, max_hits=256)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_single_surfel_scene():
    from paper_2601_23065_amd.api import BVH, Params, trace_rays
    s = sg.cloud_scene(1, seed=3)
    s.pos[:] = 0
    s.rot[:] = np.array([[1.0], [0.0], [0.0], [0.0]], dtype=np.float32)
    gs = gpu_scene(s)
    bvh = BVH(gs)
    assert bvh.info().root < 0
    o = torch.tensor([[0.0], [0.0], [-2.0]], device="cuda")
    d = torch.tensor([[0.0], [0.0], [1.0]], device="cuda")
    out, hits, cnt = trace_rays(bvh, gs, Params(), o, d, max_hits=4)
    assert int(cnt[0]) == 1 and int(hits[0, 0]) == 0
    assert abs(float(out[11, 0]) - float(s.opacity[0])) < 1e-6


def test_refit_after_moving_surfels_traces_like_a_fresh_build():
    """Refit (box update over the old topology) after a transform
    edit on 10% of the surfels: the tree keeps its invariants, and tracing
    through it gives bit-identical hit lists and traced quantities to a
    tree built from scratch over the moved scene."""
    from paper_2601_23065_amd.api import BVH, Params, trace_rays
    scene = sg.room_scene(30000, (4.0, 3.0, 2.5), 5, seed=8)
    gs = gpu_scene(scene)
    bvh = BVH(gs)
    rng = np.random.default_rng(41)
    moved = scene.copy()
    idx = rng.choice(scene.n, scene.n // 10, replace=False)
    moved.pos[:, idx] += rng.normal(0.0, 0.05, (3, idx.size)).astype(np.float32)
    q = rng.normal(size=(4, idx.size)).astype(np.float32)
    moved.rot[:, idx] = q / np.linalg.norm(q, axis=0, keepdims=True)
    gs2 = gpu_scene(moved)
    bvh.refit(gs2)
    fresh = BVH(gs2)

    n = scene.n
    info, nodes, perm = _nodes(bvh, n)
    boxes = nodes[:, :12].view(np.float32).reshape(-1, 2, 6)
    kids = nodes[:, 12:14]
    for i in range(max(n - 1, 1)):
        for c in range(2):
            k = kids[i, c]
            if k >= 0:
                child = boxes[k]
                assert np.all(child[:, :3] >= boxes[i, c, :3]) and np.all(child[:, 3:] <= boxes[i, c, 3:])

    O, D = sg.random_rays(moved, 3000, seed=42)
    O, D = torch.from_numpy(O).cuda(), torch.from_numpy(D).cuda()
    a = trace_rays(bvh, gs2, Params(), O, D, max_hits=256)
    b = trace_rays(fresh, gs2, Params(), O, D, max_hits=256)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    moved_hits = np.isin(a[1].cpu().numpy(), idx).sum()
    print(f"hits on moved surfels: {moved_hits}")
    assert moved_hits > 0
