"""The octree and interaction lists built by the HIP kernels (option tree = "gpu").

* against the oracle's plain tree (open boundary): the point orders equal the
  oracle's Morton order, every box (level, anchor) holds the same points and
  has the same leaf flag, and every U, V, W, X list holds the same boxes once
  the library's pruning is applied to the oracle's lists (entries whose box
  holds no sources, lists of boxes without targets);
* against the host builder (tree = "host"), which follows the same rules:
  every array equal, entry for entry, at the 1M-point clustered workload,
  with separate SL / DL / target sets, triply periodic trees (image shifts),
  learned per-leaf capacities and degenerate inputs (coincident points down
  to the deepest level);
* the evaluation pass on either tree gives bit-identical results.
"""
import numpy as np
import pytest
import torch

from oracle import kifmm
from paper_2010_15155_amd import FMM, workloads as W
from paper_2010_15155_amd.predictor import load_weights

pytestmark = pytest.mark.gpu

ARRAYS = ["box", "perm_sl", "perm_dl", "perm_trg"] + [n + s for n in "UVWX" for s in ("", "_off")]


def _cuda(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _tree(kernel, sl, dl, trg, cap, how, p=6, bc="open", fmm=None):
    f = fmm or FMM()
    f.set_option("tree", how)
    f.set_points(kernel, sl, dl, trg, p=p, leaf_cap=cap, bc=bc)
    return f.tree()


def _lib_view(tr):
    box = tr["box"]
    key = [tuple(int(v) for v in box[b, :4]) for b in range(len(box))]
    perms = [tr["perm_sl"], tr["perm_dl"], tr["perm_trg"]]
    idx = {key[b]: [np.sort(perms[k][box[b, 6 + 2 * k]:box[b, 7 + 2 * k]]) for k in range(3)]
           for b in range(len(box))}
    leaf = {key[b]: bool(box[b, 5]) for b in range(len(box))}
    lists = {}
    for name in "UVWX":
        off, ent = tr[name + "_off"], tr[name]
        d = {}
        for b in range(len(box)):
            e = ent[off[b]:off[b + 1]]
            if len(e) == 0:
                continue
            assert np.all(e[:, 1:] == 0)                 # open boundary: no images
            assert np.all(np.diff(e[:, 0]) > 0)          # ordered by box, no repeats
            d[key[b]] = sorted(key[a] for a in e[:, 0])
        lists[name] = d
    return idx, leaf, lists


def _oracle_view(T):
    key = {b: (int(T.level[b]),) + tuple(int(v) for v in T.anchor[b]) for b in range(T.nbox)}
    nsrc = {b: len(T.idx[b][0]) + len(T.idx[b][1]) for b in range(T.nbox)}
    ntrg = {b: len(T.idx[b][2]) for b in range(T.nbox)}
    lists = {}
    for name, L in (("U", T.U), ("V", T.V), ("W", T.W), ("X", T.X)):
        d = {}
        for b, ents in L.items():
            if ntrg[b] == 0:
                continue
            s = sorted(key[a] for a in ents if nsrc[a] > 0)
            if s:
                d[key[b]] = s
        lists[name] = d
    idx = {key[b]: [np.sort(np.asarray(T.idx[b][k], dtype=np.int64)) for k in range(3)] for b in range(T.nbox)}
    leaf = {key[b]: bool(T.is_leaf[b]) for b in range(T.nbox)}
    return idx, leaf, lists


def _oracle_cases():
    rng = np.random.default_rng(77)
    c = rng.uniform(0.25, 0.75, (3, 3))
    clus = lambda n, s: W.gaussian_mixture_points(rng, n, c, s)
    same = clus(3000, 0.06)
    pile = np.concatenate([np.full((40, 3), 0.3 + 2.0 ** -30), rng.random((60, 3))])
    return {
        "separate_sets": ("PVel", rng.random((1200, 3)), clus(2000, 0.05), clus(1600, 0.08), 30),
        "aliased": ("Stokeslet", same, None, same, 25),
        "coincident": ("Stokeslet", pile, None, pile, 10),
        "one_point": ("Stokeslet", np.array([[0.5, 0.25, 0.75]]), None, np.array([[0.5, 0.25, 0.75]]), 1),
    }


@pytest.mark.parametrize("case", list(_oracle_cases()))
def test_gpu_tree_matches_oracle(case):
    kernel, sl, dl, trg, cap = _oracle_cases()[case]
    print("tree vs oracle:", case, flush=True)
    xs = [_cuda(sl), _cuda(dl), _cuda(trg)]
    if trg is sl:
        xs[2] = xs[0]
    tr = _tree(kernel, xs[0], xs[1], xs[2], cap, "gpu")
    for name, a in (("perm_sl", sl), ("perm_dl", dl), ("perm_trg", trg)):
        if a is not None:
            assert np.array_equal(tr[name], kifmm.morton_order(a, (0, 0, 0), 1.0)), name
    T = kifmm.Tree(sl, dl, trg, (0, 0, 0), 1.0, cap)
    gi, gl, gL = _lib_view(tr)
    oi, ol, oL = _oracle_view(T)
    assert gi.keys() == oi.keys()
    assert gl == ol
    for k in gi:
        for s in range(3):
            assert np.array_equal(gi[k][s], oi[k][s]), (k, s)
    for name in "UVWX":
        assert gL[name] == oL[name], name
    if case == "coincident":
        assert tr["box"][:, 0].max() == 20


def _equal(a, b):
    for n in ARRAYS:
        assert a[n].shape == b[n].shape and np.array_equal(a[n], b[n]), n


def test_gpu_tree_equals_host_tree_1m_clustered():
    d = W.clustered_rpy(1_048_576, 201)
    x = _cuda(d["xyz"])
    for cap in (2000, 300):
        print("tree gpu vs host: 1M clustered, leaf_cap", cap, flush=True)
        g = _tree("Stokeslet", x, None, x, cap, "gpu", p=8)
        h = _tree("Stokeslet", x, None, x, cap, "host", p=8)
        _equal(g, h)
        assert len(g["V"]) > 100_000 and len(g["W"]) > 0 and len(g["X"]) > 0


def test_gpu_tree_equals_host_tree_separate_sets():
    rng = np.random.default_rng(5)
    c = rng.uniform(0.2, 0.8, (5, 3))
    sl = W.gaussian_mixture_points(rng, 60_000, c, 0.05)
    dl = W.gaussian_mixture_points(rng, 90_000, c, 0.02)
    trg = rng.random((70_000, 3))
    print("tree gpu vs host: separate sets", flush=True)
    g = _tree("PVel", _cuda(sl), _cuda(dl), _cuda(trg), 150, "gpu")
    h = _tree("PVel", _cuda(sl), _cuda(dl), _cuda(trg), 150, "host")
    _equal(g, h)
    # DL sources only
    g = _tree("PVel", None, _cuda(dl), _cuda(trg), 150, "gpu")
    h = _tree("PVel", None, _cuda(dl), _cuda(trg), 150, "host")
    _equal(g, h)


@pytest.mark.parametrize("n,cap", [(40, 3), (5000, 20), (200_000, 500)])
def test_gpu_tree_equals_host_tree_periodic(n, cap):
    rng = np.random.default_rng(n)
    # points outside the box too: the periodic plan wraps them
    x = _cuda(rng.uniform(-0.5, 1.5, (n, 3)))
    print("tree gpu vs host: periodic", n, cap, flush=True)
    g = _tree("LapPGrad", x, x, x, cap, "gpu", bc="PXYZ")
    h = _tree("LapPGrad", x, x, x, cap, "host", bc="PXYZ")
    _equal(g, h)
    assert np.any(g["U"][:, 1:] != 0) and np.any(g["V"][:, 1:] != 0)


@pytest.mark.parametrize("n,cap", [(40, 3), (5000, 20), (200_000, 500)])
def test_gpu_tree_equals_host_tree_doubly_periodic(n, cap):
    rng = np.random.default_rng(n + 1)
    # x and y outside the box too (wrapped), z inside it (open)
    x = rng.uniform(-0.5, 1.5, (n, 3))
    x[:, 2] = rng.random(n)
    x = _cuda(x)
    print("tree gpu vs host: doubly periodic", n, cap, flush=True)
    g = _tree("Stokeslet", x, None, x, cap, "gpu", bc="PXY")
    h = _tree("Stokeslet", x, None, x, cap, "host", bc="PXY")
    _equal(g, h)
    ents = np.concatenate([g[k] for k in "UVWX"])
    assert np.all(ents[:, 3] == 0) and np.any(ents[:, 1:3] != 0)


def test_gpu_tree_equals_host_tree_coincident_points():
    rng = np.random.default_rng(9)
    x = np.concatenate([np.full((3000, 3), 0.625), rng.random((20_000, 3))])
    xd = _cuda(x)
    print("tree gpu vs host: coincident points", flush=True)
    g = _tree("Stokeslet", xd, None, xd, 100, "gpu")
    h = _tree("Stokeslet", xd, None, xd, 100, "host")
    _equal(g, h)
    assert g["box"][:, 0].max() == 20


def test_gpu_tree_equals_host_tree_learned_capacities():
    d = W.mixture(903, (300_000, 300_000))
    x = _cuda(d["xyz"])
    trees = {}
    for how in ("gpu", "host"):
        print("tree gpu vs host: learned plan,", how, flush=True)
        f = FMM()
        f.set_predictor(load_weights())
        trees[how] = _tree("Stokeslet", x, None, x, 0, how, p=0, fmm=f)
        assert sum(1 for c in f.learned_info()["cap_hist"] if c > 0) > 1
    _equal(trees["gpu"], trees["host"])


def test_results_identical_on_either_tree():
    d = W.clustered_rpy(200_000, 7)
    x, fb = _cuda(d["xyz"]), _cuda(np.concatenate([d["f"], d["b"][:, None]], 1))
    outs = {}
    for how in ("gpu", "host"):
        print("RPY evaluation on the", how, "tree", flush=True)
        f = FMM()
        f.set_option("tree", how)
        outs[how] = f.evaluate("RPY", sl_xyz=x, sl_val=fb, trg_xyz=x, p=6, leaf_cap=400).clone()
    assert torch.equal(outs["gpu"], outs["host"])


@pytest.mark.parametrize("how", ["gpu", "host"])
def test_point_checks(how):
    from paper_2010_15155_amd import StkfmmError
    rng = np.random.default_rng(3)
    x = rng.random((5000, 3))
    f = FMM()
    f.set_option("tree", how)
    bad = x.copy()
    bad[1234, 1] = np.nan
    with pytest.raises(StkfmmError) as ei:
        f.set_points("Stokeslet", _cuda(x), None, _cuda(bad), p=6, leaf_cap=100)
    assert ei.value.status == "E_ARG" and "trg_xyz" in str(ei.value)
    out = x.copy()
    out[4321, 2] = 1.0                           # the upper face is outside the half-open box
    with pytest.raises(StkfmmError) as ei:
        f.set_points("Stokeslet", _cuda(out), None, _cuda(x), p=6, leaf_cap=100)
    assert ei.value.status == "E_DOMAIN" and "sl_xyz" in str(ei.value)
    # periodic plans wrap instead
    f.set_points("LapPGrad", _cuda(out), None, _cuda(x), p=6, leaf_cap=100, bc="PXYZ")


def test_leaf_features_after_a_gpu_tree_plan():
    d = W.mixture(905, (200_000, 200_000))
    x = _cuda(d["xyz"])
    feats = {}
    for how in ("gpu", "host"):
        f = FMM()
        f.set_option("tree", how)
        f.set_points("Stokeslet", x, None, x, p=8, leaf_cap=2000)
        feats[how] = f.leaf_features()
    assert np.array_equal(feats["gpu"][0], feats["host"][0])
    assert np.array_equal(feats["gpu"][1], feats["host"][1])
