"""GPU tests of the autotuner: launch shapes only permute work over
workgroups, so every tuning table must give the same bits; the tuned table
is applied and can be re-applied to a fresh plan."""
import numpy as np
import pytest

from paper_1507_04789_amd import MRA_SYNC, Plan
from paper_1507_04789_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = ["identity", "grouped", "chunked"]


def test_autotune_keeps_results_bitwise():
    w = wl.clustered(n=32768, M=4, r=64)
    print("tuning case: clustered n=%d M=%d" % (len(w.z), w.M), flush=True)
    p = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, flags=MRA_SYNC)
    z = torch.tensor(w.z, device="cuda")
    th = torch.tensor(w.theta, dtype=torch.float64, device="cuda").reshape(1, 3)
    ll0, g0 = p.loglik_grad(z, th)
    table = p.autotune(z, th, reps=1)
    assert table["families"].keys() == p.tuning()["families"].keys()
    ll1, g1 = p.loglik_grad(z, th)
    assert torch.equal(ll0, ll1) and torch.equal(g0, g1)
    # every family forced to one shape, and the large-leaf cut varied
    for k, shape in enumerate(SHAPES):
        t = p.tuning()
        for f in t["families"]:
            t["families"][f] = shape
        t["big_leaf_tiles"] = [0, 2, 4][k]
        t["side_solves"] = [0, 3, w.M + 2][k]   # main stream; forked after the top level; at the end
        p.set_tuning(t)
        ll2, g2 = p.loglik_grad(z, th)
        assert torch.equal(ll0, ll2) and torch.equal(g0, g2), shape
    q = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, flags=MRA_SYNC)
    q.set_tuning(table)
    ll3, g3 = q.loglik_grad(z, th)
    assert torch.equal(ll0, ll3) and torch.equal(g0, g3)


def test_leaf_solve_fork_stages_bitwise():
    """The reverse pass's leaf solves forked at every kind of stage (main
    stream, before and after the leaf reduction, after a posterior level,
    after a reverse posterior level, past the last stage), eagerly and in a
    captured graph, with the data gradient: the same bits each time."""
    from paper_1507_04789_amd import MRA_GRAPH
    w = wl.clustered(n=32768, M=4, r=64)
    M = w.M
    print("fork-stage case: clustered n=%d M=%d" % (len(w.z), M), flush=True)
    z = torch.tensor(w.z, device="cuda")
    th = torch.tensor(w.theta, dtype=torch.float64, device="cuda").reshape(1, 3)
    ref = None
    for flags in (MRA_SYNC, MRA_SYNC | MRA_GRAPH):
        p = Plan(w.locs, M=M, J=w.J, r=w.r, cov=w.cov, flags=flags)
        for s in [0, 1, 2, M, M + 2, M + 3, 2 * M + 1, 2 * M + 6]:
            t = p.tuning()
            t["side_solves"] = s
            p.set_tuning(t)
            out = p.loglik_grad_data(z, th)
            if ref is None:
                ref = [o.clone() for o in out]
            for a, b in zip(out, ref):
                assert torch.equal(a, b), (flags, s)
