"""Host-side checks of the C ABI (no GPU needed): every declared symbol is
exported, plans build and reject bad input, and the library's geometry
agrees bit for bit with the oracle's independent implementation."""
import math
import re
import os

import numpy as np
import pytest

from oracle.geometry import Geometry
from paper_1507_04789_amd import _lib, Plan, MRAError
from paper_1507_04789_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "mra.h")).read()
    declared = set(re.findall(r"\b(mra_[a-z_]+)\s*\(", hdr))
    assert declared == set(_lib.SYMBOLS)
    L = _lib.lib()
    for name in declared:
        assert hasattr(L, name)


@pytest.mark.parametrize("d,J,M,r,n", [(2, 4, 3, 16, 4096), (2, 4, 5, 64, 20000), (1, 2, 6, 4, 700),
                                       (1, 3, 4, 2, 500), (2, 4, 0, 16, 300)])
def test_geometry_matches_oracle(d, J, M, r, n):
    g0 = np.random.default_rng(M + 10 * d)
    locs = g0.random((n, d))
    locs[:5] = 0.5
    locs[5] = 1.0
    locs[6] = 0.0
    p = Plan(locs, M=M, J=J, r=r, cov="matern32")
    perm, off, kn = p.geometry()
    og = Geometry(locs, d, M, J, r)
    assert (perm == og.perm).all()
    assert (off == og.offsets).all()
    for m in range(M):
        assert np.array_equal(kn[m], og.knots[m])   # bitwise


@pytest.mark.parametrize("Jl,rl,adaptive", [((2, 2, 4, 8), (16, 9, 9, 4), False), ((2, 2, 4, 8), (16, 9, 9, 4), True),
                                            ((4, 16), (64, 16), True), ((8, 4, 2), (4, 4, 4), True)])
def test_mixed_and_adaptive_geometry_matches_oracle(Jl, rl, adaptive):
    """Level-dependent J_m, r_m and adaptive splits: the library's partition
    (leaf order and CSR offsets) and default knots equal the oracle's bit for
    bit, also for prediction locations (their leaves follow the same splits)."""
    w = wl.clustered(n=20000, M=len(Jl))
    M = len(Jl)
    pred = np.random.default_rng(4).random((500, 2))
    p = Plan(w.locs, M=M, J=4, r=4, cov=w.cov, J_levels=Jl, r_levels=rl, adaptive=adaptive, pred=pred)
    perm, off, kn = p.geometry()
    og = Geometry(w.locs, 2, M, 4, 4, J_levels=Jl, r_levels=rl, adaptive=adaptive)
    assert (perm == og.perm).all() and (off == og.offsets).all()
    for m in range(M):
        assert np.array_equal(kn[m], og.knots[m])
    assert p.info["n_leaves"] == og.nreg[M]
    if adaptive:   # flatter leaves than equal-area splits of the clustered scatter
        eq = Geometry(w.locs, 2, M, 4, 4, J_levels=Jl, r_levels=rl)
        assert np.diff(og.offsets).max() < np.diff(eq.offsets).max()


def test_clustered_geometry_matches_oracle():
    w = wl.clustered(n=32768, M=5)
    p = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov)
    perm, off, _ = p.geometry()
    og = Geometry(w.locs, 2, w.M, w.J, w.r)
    assert (perm == og.perm).all() and (off == og.offsets).all()
    assert p.info["max_leaf"] == np.diff(og.offsets).max()


def test_explicit_knots_roundtrip():
    g0 = np.random.default_rng(3)
    locs = g0.random((100, 2))
    kn = [g0.random((4 ** m, 9, 2)) for m in range(2)]
    p = Plan(locs, M=2, J=4, r=9, cov="exponential", knots=kn)
    _, _, got = p.geometry()
    assert all(np.array_equal(a, b) for a, b in zip(got, kn))


@pytest.mark.parametrize("bad", [
    dict(M=3, J=4, r=15),          # default 2-D knots need a square r
    dict(M=3, J=3, r=16),          # d = 2 needs J in {1, 2, 4, 8, 16}
    dict(M=3, J=4, r=65),          # r above the tile
    dict(M=12, J=4, r=16),         # too many levels
])
def test_rejects_bad_config(bad):
    locs = np.random.default_rng(0).random((50, 2))
    with pytest.raises(MRAError) as e:
        Plan(locs, cov="matern32", **bad)
    assert e.value.status == _lib.MRA_EINVAL


def test_rejects_out_of_box_and_nan():
    locs = np.random.default_rng(0).random((50, 2))
    locs[3] = [1.5, 0.2]
    with pytest.raises(MRAError):
        Plan(locs, M=2, J=4, r=4, cov="matern32")
    locs[3] = [np.nan, 0.2]
    with pytest.raises(MRAError):
        Plan(locs, M=2, J=4, r=4, cov="matern32")


def test_flop_model_counts():
    w = wl.small_uniform()
    p = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov)
    assert p.info["n_leaves"] == 64 and p.info["n_regions"] == 85
    assert p.info["flops_grad"] > p.info["flops_loglik"] > 0


def test_binding_rejects_narrow_tensors():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(3)
    p = Plan(g.random((200, 2)), M=1, J=4, r=4, cov="exponential")
    with pytest.raises(TypeError):
        p.loglik(torch.zeros(200, dtype=torch.float32), np.zeros(3))
    with pytest.raises(TypeError):
        p.loglik_grad(np.zeros(200), torch.zeros(1, 3, dtype=torch.float32))


def test_rejects_unknown_flags():
    g = np.random.default_rng(4)
    with pytest.raises(MRAError):
        Plan(g.random((100, 2)), M=1, J=4, r=4, cov="exponential", flags=64)


def test_tuning_table_roundtrip():
    g = np.random.default_rng(5)
    p = Plan(g.random((500, 2)), M=2, J=4, r=9, cov="exponential")
    t = p.tuning()
    assert t["big_leaf_tiles"] == 3 and t["side_solves"] == 2 + 2 and set(t["families"].values()) == {"default"}
    t["families"]["leaf_rows"] = "identity"
    t["families"]["rT_leaf"] = "chunked"
    t["big_leaf_tiles"] = 0
    t["side_solves"] = 1
    p.set_tuning(t)
    u = p.tuning()
    assert u["families"]["leaf_rows"] == "identity" and u["families"]["rT_leaf"] == "chunked"
    assert u["big_leaf_tiles"] == 0 and u["side_solves"] == 1
    with pytest.raises(MRAError):
        p.set_tuning({"side_solves": -1})
    with pytest.raises(MRAError):
        p.set_tuning({"families": {"post": "sideways"}})
    with pytest.raises(MRAError):
        p.set_tuning({"big_leaf_tiles": -2})
