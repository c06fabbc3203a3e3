"""The entry point that allocates nothing (mra_loglik_grad_noalloc), called
through the C ABI: its work arena is the library's own scratch array, its
plan has only the geometry bound, and it must give what mra_loglik_grad
gives on a fully bound plan (the same kernels, so the same bits), on two
calls in a row, the second with a smaller input, which finds the first
call's contents in the shared array.  Sizes beyond the array's limit are
refused before anything is launched."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_1507_04789_amd import Plan, _lib
from paper_1507_04789_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _th(s2, k, t2):
    return [math.log(s2), math.log(k), math.log(t2)]


def _reference(locs, z, ths, **kw):
    """mra_loglik_grad on a plan with both arenas bound."""
    p = Plan(locs, max_theta=len(ths), **kw)
    p.bind("cuda:0")
    ll, g = p.loglik_grad(torch.tensor(z, device="cuda:0"), torch.tensor(ths, dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()
    return ll.cpu().numpy(), g.cpu().numpy()


def _noalloc(locs, z, ths, **kw):
    """mra_loglik_grad_noalloc through ctypes on a geometry-only plan."""
    p = Plan(locs, max_theta=len(ths), **kw)
    p.bind("cuda:0", work=False)
    assert p._work is None
    zt = torch.tensor(np.asarray(z, dtype=np.float64), device="cuda:0")
    tt = torch.tensor(ths, dtype=torch.float64, device="cuda:0")
    assert zt.dtype == torch.float64 and tt.shape == (len(ths), 3)
    ll = torch.full((len(ths),), float("nan"), dtype=torch.float64, device="cuda:0")
    g = torch.full((len(ths), 3), float("nan"), dtype=torch.float64, device="cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    # the ordinary calls refuse a plan without a work arena
    assert _lib.lib().mra_loglik(p._h, zt.data_ptr(), tt.data_ptr(), len(ths), ll.data_ptr(), st) == _lib.MRA_ESTATE
    s = _lib.lib().mra_loglik_grad_noalloc(p._h, zt.data_ptr(), tt.data_ptr(), len(ths), ll.data_ptr(),
                                           g.data_ptr(), st)
    assert s == _lib.MRA_OK, s
    torch.cuda.synchronize()
    return ll.cpu().numpy(), g.cpu().numpy()


def _compare(got, ref):
    (ll, g), (rll, rg) = got, ref
    assert np.isfinite(ll).all() and np.isfinite(g).all()
    assert (np.abs(ll - rll) <= 1e-10 * np.abs(rll)).all(), (ll, rll)
    assert (np.abs(g - rg) <= 1e-6 * np.abs(rg)).all(), (g, rg)
    # the same kernels in the same order: bit-identical
    assert np.array_equal(ll, rll) and np.array_equal(g, rg), (ll - rll, g - rg)


def test_noalloc_two_calls_second_smaller():
    # first call: the small uniform workload (n = 4096, exponential, M = 3,
    # r = 16) at two parameter vectors, about 144 MB of the 256 MiB array
    w = wl.small_uniform()
    ths = [list(map(float, w.theta)), _th(0.8, 0.1, 0.02)]
    kw = dict(M=w.M, J=w.J, r=w.r, cov=w.cov)
    print("noalloc call 1: n=%d M=%d r=%d, 2 thetas" % (len(w.z), w.M, w.r), flush=True)
    _compare(_noalloc(w.locs, w.z, ths, **kw), _reference(w.locs, w.z, ths, **kw))
    # second call: a smaller plan (n = 1500, Matern, M = 2, r = 9) at one
    # vector, on the array the first call left behind
    g = np.random.default_rng(31)
    locs = g.random((1500, 2))
    z = g.standard_normal(1500)
    th2 = [_th(1.2, 0.15, 0.03)]
    kw2 = dict(M=2, J=4, r=9, cov="matern32")
    print("noalloc call 2: n=1500 M=2 r=9, 1 theta", flush=True)
    _compare(_noalloc(locs, z, th2, **kw2), _reference(locs, z, th2, **kw2))


def test_noalloc_refuses_beyond_limit():
    # n = 16384, M = 4, r = 16 needs about 320 MB per parameter vector
    g = np.random.default_rng(32)
    locs = g.random((16384, 2))
    p = Plan(locs, M=4, J=4, r=16, cov="matern32")
    assert p.work_bytes > _lib.NOALLOC_MAX_BYTES
    p.bind("cuda:0", work=False)
    z = torch.zeros(16384, dtype=torch.float64, device="cuda:0")
    th = torch.tensor([_th(1.0, 0.1, 0.01)], dtype=torch.float64, device="cuda:0")
    ll = torch.empty(1, dtype=torch.float64, device="cuda:0")
    gr = torch.empty(1, 3, dtype=torch.float64, device="cuda:0")
    s = _lib.lib().mra_loglik_grad_noalloc(p._h, z.data_ptr(), th.data_ptr(), 1, ll.data_ptr(), gr.data_ptr(),
                                           torch.cuda.current_stream().cuda_stream)
    assert s == _lib.MRA_ENOMEM
