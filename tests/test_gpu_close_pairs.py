"""GPU parity for distinct points of different leaves that lie closer than
the Stokeslet P2P's leaf-relative FP32 positions resolve (Sec. III.A: the
near field is summed directly, so such a pair is the largest term of both
points' velocities).

The plan finds such pairs and then forms r from the hi/lo coordinates, whose
difference keeps the pair's separation; ordinary inputs keep the faster
leaf-relative form.
"""
import numpy as np
import pytest
import torch

from oracle import direct
from oracle.stokes_dp import stokeslet_dp
from paper_2010_15155_amd import FMM

pytestmark = pytest.mark.gpu


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def fmm():
    f = FMM()
    yield f
    f.close()


@pytest.mark.parametrize("gap", [1e-9, 2e-7])
def test_pair_across_leaf_faces(fmm, gap):
    rng = np.random.default_rng(31)
    x = rng.random((2000, 3))
    # x = 0.5 is a face of every level's boxes
    x[0] = (0.5 - gap / 2, 0.31, 0.72)
    x[1] = (0.5 + gap / 2, 0.31, 0.72)
    f = rng.standard_normal((len(x), 3))
    print("close pair across x = 0.5, gap", gap, flush=True)
    out = fmm.evaluate("Stokeslet", sl_xyz=cu(x), sl_val=cu(f), trg_xyz=cu(x), p=8,
                       leaf_cap=32).cpu().numpy()
    st = fmm.stats()
    assert st["depth"] >= 3 and st["p2p_exact_r"] == 1
    ref = direct.stokeslet(x, f, x)
    e_pair, e_all = rel(out[:2], ref[:2]), rel(out, ref)
    print("  pair", e_pair, "all", e_all, flush=True)
    assert e_pair < 1e-6 and e_all < 1e-5


def test_pair_across_periodic_face(fmm):
    rng = np.random.default_rng(32)
    x = rng.random((3000, 3))
    x[0] = (2e-10, 0.45, 0.4)                   # the pair is 5e-10 apart through x = 0 == 1
    x[1] = (1.0 - 3e-10, 0.45, 0.4)
    f = rng.standard_normal((len(x), 3))
    f -= f.mean(axis=0)
    print("close pair across the periodic face, PXY", flush=True)
    out = fmm.evaluate("Stokeslet", sl_xyz=cu(x), sl_val=cu(f), trg_xyz=cu(x), p=8, leaf_cap=40,
                       bc="PXY").cpu().numpy()
    assert fmm.stats()["p2p_exact_r"] == 1
    idx = np.r_[0, 1, np.arange(2, len(x), 15)]
    ref = stokeslet_dp(x, f, x[idx])
    e_pair, e_all = rel(out[:2], ref[:2]), rel(out[idx], ref)
    print("  pair", e_pair, "sampled", e_all, flush=True)
    assert e_pair < 1e-6 and e_all < 1e-5


def test_ordinary_points_keep_leaf_relative_form(fmm):
    rng = np.random.default_rng(33)
    x = rng.random((20000, 3))
    f = rng.standard_normal((len(x), 3))
    fmm.evaluate("Stokeslet", sl_xyz=cu(x), sl_val=cu(f), trg_xyz=cu(x), p=6, leaf_cap=64)
    assert fmm.stats()["p2p_exact_r"] == 0
