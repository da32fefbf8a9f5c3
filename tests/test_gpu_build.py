"""GPU LBVH build vs the oracle: Morton keys, sort order and radix-tree topology
bit-exact; leaf boxes conservative and tight against the FP64 3-sigma boxes;
internal boxes the exact union of their children; compressed four-wide records
list the grandchildren of each node with outward-rounded boxes; repeated builds
identical."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2311_16043_amd import Gaussians, TraceParams, build_bvh, refit_bvh, trace_rays
from workloads import scenes

from _parity import check_vis, oracle_lbvh

pytestmark = pytest.mark.gpu


def _build(scene):
    g = Gaussians.from_scene(scene)
    bvh = build_bvh(g)
    torch.cuda.synchronize()
    return g, bvh, bvh.arrays()


def check_nodes4(A):
    """Compressed four-wide records: slot kinds and indices are the
    grandchildren of each node (a leaf child keeps its own slot, the next is
    empty); every decoded plane O + q step lies outside the child's binary box
    by at least the margin eta and by at most eta plus one step."""
    W = A["nodes4"]
    m = W.shape[0]
    assert np.all(W[:, 12:16] == 0)
    meta = W[:, 3]
    kind = np.stack([(meta >> (24 + 2 * j)) & 3 for j in range(4)], 1)
    idx = np.stack([W[:, 10].view(np.int32), W[:, 10].view(np.int32) + 1,
                    W[:, 11].view(np.int32), W[:, 11].view(np.int32) + 1], 1)
    exp_kind = np.zeros((m, 4), np.uint32)
    exp_idx = np.zeros((m, 4), np.int64)
    boxes = np.zeros((m, 4, 6), np.float64)
    for side, (ch, cbox) in enumerate(((A["left"], A["left_box"]), (A["right"], A["right_box"]))):
        leaf = ch < 0
        s0, s1 = 2 * side, 2 * side + 1
        exp_kind[leaf, s0] = 3
        exp_idx[leaf, s0] = ~ch[leaf]
        boxes[leaf, s0] = cbox[leaf]
        inner = np.nonzero(~leaf)[0]
        c = ch[inner]
        lc, rc = A["left"][c], A["right"][c]
        exp_kind[inner, s0] = np.where(lc < 0, 3, 1)
        exp_kind[inner, s1] = np.where(rc < 0, 3, 1)
        exp_idx[inner, s0] = np.where(lc < 0, ~lc, lc)
        exp_idx[inner, s1] = np.where(rc < 0, ~rc, rc)
        boxes[inner, s0] = A["left_box"][c]
        boxes[inner, s1] = A["right_box"][c]
    assert np.array_equal(kind, exp_kind), "slot kinds differ from the grandchildren"
    used = exp_kind != 0
    assert np.array_equal(idx[used], exp_idx[used]), "slot indices differ from the grandchildren"
    root = A["header"][6:12].astype(np.float64)
    eta = (np.abs(root).max() + np.linalg.norm(root[3:] - root[:3]) + 1.0) * 2.0 ** -20
    O = W[:, 0:3].view(np.float32).astype(np.float64)
    step = np.stack([2.0 ** (((meta >> (8 * a)) & 0xFF).astype(np.float64) - 127) for a in range(3)], 1)
    for a in range(3):
        qlo = np.stack([(W[:, 4 + a] >> (8 * j)) & 0xFF for j in range(4)], 1).astype(np.float64)
        qhi = np.stack([(W[:, 7 + a] >> (8 * j)) & 0xFF for j in range(4)], 1).astype(np.float64)
        dlo = O[:, a:a + 1] + qlo * step[:, a:a + 1]
        dhi = O[:, a:a + 1] + qhi * step[:, a:a + 1]
        lo, hi = boxes[:, :, a], boxes[:, :, 3 + a]
        tol = 1e-12 * (np.abs(lo) + np.abs(hi) + 1.0) + np.abs(O[:, a:a + 1]) * 2.0 ** -23
        assert np.all((dlo <= lo - eta + tol)[used]) and np.all((dhi >= hi + eta - tol)[used]), \
            f"a decoded plane cuts into its child box (axis {a})"
        slack = eta + step[:, a:a + 1] + tol
        assert np.all((lo - dlo <= slack)[used]) and np.all((dhi - hi <= slack)[used]), \
            f"decoded planes not tight (axis {a})"


def check_build(scene, label=""):
    n = scene["mean"].shape[0]
    print(f"[build {label}] n={n}", flush=True)
    g, bvh, A = _build(scene)
    O = oracle_lbvh(scene)
    assert np.array_equal(A["header"][0:3], O["lo"]) and np.array_equal(A["header"][3:6], O["hi"])
    assert np.array_equal(A["keys"], O["keys"][O["order"]]), "sorted Morton keys differ"
    assert np.array_equal(A["perm"].astype(np.int64), O["order"]), "sort permutation differs"
    if n > 1:
        assert np.array_equal(A["left"], O["left"]), "left children differ"
        assert np.array_equal(A["right"], O["right"]), "right children differ"
    assert np.array_equal(A["parent"], O["parent"]), "parents differ"
    # leaf records carry the source index and opacity in sorted order
    rec = A["leaf_records"]
    assert np.array_equal(rec[:, 11].view(np.int32).astype(np.int64), O["order"])
    assert np.array_equal(rec[:, 3], scene["opacity"][O["order"]])
    assert np.array_equal(rec[:, 0:3], scene["mean"][O["order"]])
    # whitening rows 0 and 1 as stored, row 2 as the tracer rebuilds it
    # (s0 s1 / s2 times row 0 x row 1), against the FP64 W = diag(1/s) R^T
    w0, w1 = rec[:, 4:7].astype(np.float64), rec[:, 8:11].astype(np.float64)
    w2 = rec[:, 7:8].astype(np.float64) * np.cross(w0, w1)
    for k in np.linspace(0, n - 1, min(n, 200)).astype(np.int64):
        i = O["order"][k]
        Wo = oracle.whitening(scene["quat"][i], scene["log_scale"][i])
        Wg = np.stack([w0[k], w1[k], w2[k]])
        assert np.allclose(Wg, Wo, rtol=0, atol=2e-6 * np.abs(Wo).max()), (k, Wg, Wo)
    # leaf boxes: contain the FP64 3-sigma box, and are tight
    llo, lhi = oracle.leaf_boxes(scene)
    olo, ohi = llo[O["order"]], lhi[O["order"]]
    glo = A["leaf_boxes"][:, 0:3].astype(np.float64)
    ghi = A["leaf_boxes"][:, 3:6].astype(np.float64)
    assert np.all(glo <= olo) and np.all(ghi >= ohi), "a leaf box cuts into the 3-sigma support"
    # widening: 2^-12 relative plus 2^-20 of the scene scale (max |coord| + diagonal + 1)
    lo_m, hi_m = O["lo"].astype(np.float64), O["hi"].astype(np.float64)
    scale = max(np.abs(lo_m).max(), np.abs(hi_m).max()) + np.linalg.norm(hi_m - lo_m) + 1.0
    slack = 0.5 * (ohi - olo) * 1e-3 + 2.0 ** -19 * scale + 1e-6 * np.abs(olo)
    assert np.all(olo - glo <= slack) and np.all(ghi - ohi <= slack), "leaf boxes not tight"
    if n > 1:
        # every child slot holds the child's own box: the leaf box, or the union
        # of the internal child's two slots (exact min/max)
        lb, rb = A["left_box"], A["right_box"]
        node_box = np.concatenate([np.minimum(lb[:, 0:3], rb[:, 0:3]), np.maximum(lb[:, 3:6], rb[:, 3:6])], 1)
        for slot, ch in ((lb, A["left"]), (rb, A["right"])):
            leaf = ch < 0
            assert np.array_equal(slot[leaf], A["leaf_boxes"][~ch[leaf]])
            assert np.array_equal(slot[~leaf], node_box[ch[~leaf]])
        root = node_box[0]
        check_nodes4(A)
    else:
        root = A["leaf_boxes"][0]
    allb = np.concatenate([A["leaf_boxes"][:, 0:3].min(0), A["leaf_boxes"][:, 3:6].max(0)])
    assert np.array_equal(root, allb) and np.array_equal(A["header"][6:12], allb)
    return g, bvh, A


def test_build_tiny_full():
    check_build(scenes.make_scene("tiny"), "tiny")


def test_build_object_small_and_ragged():
    check_build(scenes.make_object_scene(20_001, 1), "object-20001")


def test_build_multi_small():
    check_build(scenes.make_multi_object_scene(4, 5_000, 2), "multi-4x5000")


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 2047, 2048, 2049])
def test_build_edge_sizes(n):
    check_build(scenes.make_cube_cloud(n, 0), f"cube-{n}")


def test_build_duplicate_means_use_position_tiebreak():
    sc = scenes.make_cube_cloud(300, 0)
    sc["mean"][:] = sc["mean"][17]          # all keys equal
    check_build(sc, "all-equal")
    sc = scenes.make_cube_cloud(500, 0)
    sc["mean"][::2] = sc["mean"][1]         # half of them equal
    check_build(sc, "half-equal")


def test_build_planar_scene_zero_extent_axis():
    sc = scenes.make_cube_cloud(1000, 0)
    sc["mean"][:, 2] = np.float32(0.25)
    check_build(sc, "planar")


def test_build_is_deterministic():
    sc = scenes.make_object_scene(50_000, 1)
    _, _, A = _build(sc)
    for _ in range(4):
        _, _, B = _build(sc)
        for k in A:
            assert np.array_equal(A[k].view(np.uint8), B[k].view(np.uint8)), k


def test_build_object_scale_full_size():
    """Object-scale scene at its full 300,000 Gaussians."""
    check_build(scenes.make_scene("object"), "object-300k")


def test_build_multi_object_full_size():
    """Multi-object composition at its full 1.2M Gaussians: Morton, sort and
    topology bit-exact."""
    check_build(scenes.make_scene("multi"), "multi-1.2M")


def test_refit_with_unchanged_inputs_reproduces_the_build():
    sc = scenes.make_object_scene(30_000, 1)
    g, bvh, A = _build(sc)
    refit_bvh(bvh, g)
    torch.cuda.synchronize()
    B = bvh.arrays()
    for k in A:
        assert np.array_equal(A[k].view(np.uint8), B[k].view(np.uint8)), k


@pytest.mark.parametrize("n_obj,per,moved", [(4, 5_000, 2), (3, 20_001, 1)])
def test_refit_after_moving_an_object(n_obj, per, moved):
    """Scene edit (Sec. 4.3): turn and shift one object of a composition, refit
    instead of rebuilding. Order and topology stay those of the build; the
    leaf boxes are those of the moved Gaussians, every slot holds its child's
    box, the wide records cover their children, and traced visibility agrees
    with the FP64 brute force on the edited scene."""
    sc = scenes.make_multi_object_scene(n_obj, per, 2)
    print(f"[refit] {n_obj} x {per}, object {moved} moved", flush=True)
    g, bvh, A = _build(sc)
    sel = slice(moved * per, (moved + 1) * per)
    sc2 = scenes.rigid_move(sc, sel, 0.7, [0.35, -0.2, 0.15])
    g2 = Gaussians.from_scene(sc2)
    refit_bvh(bvh, g2)
    torch.cuda.synchronize()
    B = bvh.arrays()
    for k in ("keys", "perm", "left", "right", "parent"):
        assert np.array_equal(A[k], B[k]), k
    order = B["perm"].astype(np.int64)
    rec = B["leaf_records"]
    assert np.array_equal(rec[:, 0:3], sc2["mean"][order])
    llo, lhi = oracle.leaf_boxes(sc2)
    olo, ohi = llo[order], lhi[order]
    glo, ghi = B["leaf_boxes"][:, 0:3].astype(np.float64), B["leaf_boxes"][:, 3:6].astype(np.float64)
    assert np.all(glo <= olo) and np.all(ghi >= ohi), "a refitted leaf box cuts into the 3-sigma support"
    lo_m = sc2["mean"].min(0).astype(np.float64)
    hi_m = sc2["mean"].max(0).astype(np.float64)
    assert np.array_equal(B["header"][0:3], sc2["mean"].min(0)) and np.array_equal(B["header"][3:6], sc2["mean"].max(0))
    scale = max(np.abs(lo_m).max(), np.abs(hi_m).max()) + np.linalg.norm(hi_m - lo_m) + 1.0
    slack = 0.5 * (ohi - olo) * 1e-3 + 2.0 ** -19 * scale + 1e-6 * np.abs(olo)
    assert np.all(olo - glo <= slack) and np.all(ghi - ohi <= slack), "refitted leaf boxes not tight"
    lb, rb = B["left_box"], B["right_box"]
    node_box = np.concatenate([np.minimum(lb[:, 0:3], rb[:, 0:3]), np.maximum(lb[:, 3:6], rb[:, 3:6])], 1)
    for slot, ch in ((lb, B["left"]), (rb, B["right"])):
        leaf = ch < 0
        assert np.array_equal(slot[leaf], B["leaf_boxes"][~ch[leaf]])
        assert np.array_equal(slot[~leaf], node_box[ch[~leaf]])
    check_nodes4(B)
    # traced visibility on the edited scene, refit tree
    dirs = scenes.fibonacci_dirs(32, True)
    ids = scenes.sample_ray_ids(n_obj * per, 32, 2048, seed=31)
    got = trace_rays(bvh, g2, dirs, ids, TraceParams()).cpu().numpy()
    orc = oracle.trace_rays(sc2, dirs, 1, ids)
    check_vis(got, orc, label=f"refit {n_obj}x{per}")
