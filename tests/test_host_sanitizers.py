"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/host/host_checks.cpp drives the C ABI's host-only entry points; it is
linked with the plan builder and the API layer compiled with both sanitizers
(host code only: the device objects are the ordinary build's).  Two uses:

* a seeded fuzz of random plans (valid and invalid configurations, boundary,
  clustered and duplicate locations, prediction points, explicit knots),
  compute calls on unbound plans, null arguments, and a mutation fuzz of the
  tuning-table parser behind mra_set_tuning;
* the geometry cases of the ABI tests, built inside the sanitized program and
  compared bit for bit with the oracle's independent partition.

No GPU is needed; nothing here runs on one.
"""
import ctypes as C
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from oracle.geometry import Geometry
from paper_1507_04789_amd import _lib
from paper_1507_04789_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1507_04789_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitize")
EXE = os.path.join(OUT, "host_checks")
ROCM = "/opt/rocm"
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
DEVICE_OBJS = ["fwd.hip", "grad.hip", "predict.hip", "gls.hip", "predjoint.hip", "noalloc.hip"]

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
COMMON = ["-std=c++17", "-O1", "-g", "-Wall", "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1:strict_string_checks=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["LSAN_OPTIONS"] = "suppressions=" + os.path.join(ROOT, "tests", "host", "lsan.supp")
    return env


@pytest.fixture(scope="module")
def exe():
    if not (os.path.exists(CLANG) and os.path.exists(HIPCC)):
        pytest.skip("ROCm compilers not found")
    objdir = os.path.join(ROOT, "_build")
    if not all(os.path.exists(os.path.join(objdir, s + ".o")) for s in DEVICE_OBJS):
        from paper_1507_04789_amd import build
        build.build()
    os.makedirs(OUT, exist_ok=True)
    o = os.path.join(OUT, "host_checks.cpp.o")
    _run([CLANG] + COMMON + SAN + ["-c", os.path.join(ROOT, "tests", "host", "host_checks.cpp"), "-o", o])
    objs = [o]
    # the plan builder and the API layer share headers with device code:
    # host side sanitized, device side compiled as in the ordinary build
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    for src in ("plan.cpp", "api.cpp"):
        o = os.path.join(OUT, src + ".o")
        _run([HIPCC] + COMMON + ["--offload-arch=gfx950", "-x", "hip", "-Xclang", "-target-feature", "-Xclang",
                                 "-packed-fp32-ops"] + host_san + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    objs += [os.path.join(objdir, s + ".o") for s in DEVICE_OBJS]
    _run([CLANG] + SAN + ["-o", EXE] + objs + ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
                                               "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    yield EXE
    shutil.rmtree(OUT, ignore_errors=True)


def _check_clean(r):
    text = r.stdout + r.stderr
    assert "AddressSanitizer" not in text and "runtime error" not in text and "LeakSanitizer" not in text, text[-4000:]
    assert r.returncode == 0, text[-4000:]


@pytest.mark.parametrize("seed", [1, 2])
def test_fuzz_plans_and_tuning_parser(exe, seed):
    r = subprocess.run([exe, "fuzz", "300", str(seed)], capture_output=True, text=True, env=_env(), timeout=600)
    _check_clean(r)
    assert "0 failed checks" in r.stdout


def _geometry(exe, tmp_path, cfg, locs, pred=None, knots=None):
    d = cfg.d
    req = bytes(cfg) + struct.pack("<q", locs.shape[0]) + np.ascontiguousarray(locs, np.float64).tobytes()
    pred = np.zeros((0, d)) if pred is None else pred
    req += struct.pack("<q", pred.shape[0]) + np.ascontiguousarray(pred, np.float64).tobytes()
    kn = np.zeros(0) if knots is None else np.concatenate([np.asarray(k, np.float64).reshape(-1) for k in knots])
    req += struct.pack("<q", kn.size) + kn.tobytes()
    fi, fo = tmp_path / "req.bin", tmp_path / "out.bin"
    fi.write_bytes(req)
    r = subprocess.run([exe, "geometry", str(fi), str(fo)], capture_output=True, text=True, env=_env(), timeout=600)
    _check_clean(r)
    raw = fo.read_bytes()
    st = struct.unpack_from("<i", raw, 0)[0]
    if st != 0:
        return st, None
    q = 4
    info = _lib.Info.from_buffer_copy(raw[q:q + C.sizeof(_lib.Info)])
    q += C.sizeof(_lib.Info) + 16
    n, nl = locs.shape[0], info.n_leaves
    perm = np.frombuffer(raw, np.int64, n, q)
    q += 8 * n
    off = np.frombuffer(raw, np.int64, nl + 1, q)
    q += 8 * (nl + 1)
    return st, (info, perm, off, raw, q)


def _cfg(d, M, J, r, Jl=None, rl=None, adaptive=False, flags=_lib.MRA_SYNC):
    c = _lib.Config()
    c.d, c.M, c.J, c.r = d, M, J, r
    for a in range(d):
        c.lo[a], c.hi[a] = 0.0, 1.0
    c.cov, c.max_theta, c.flags = 1, 1, flags
    for m in range(M):
        c.J_level[m] = 0 if Jl is None else Jl[m]
        c.r_level[m] = 0 if rl is None else rl[m]
    c.adaptive = 1 if adaptive else 0
    return c


def _knots_from(raw, q, og):
    out = []
    for m in range(og.M):
        k = np.frombuffer(raw, np.float64, og.knots[m].size, q)
        out.append(k.reshape(og.knots[m].shape))
        q += 8 * og.knots[m].size
    return out


@pytest.mark.parametrize("d,J,M,r,n", [(2, 4, 3, 16, 4096), (1, 2, 6, 4, 700), (1, 3, 4, 2, 500),
                                       (1, 16, 2, 3, 900), (2, 4, 0, 16, 300)])
def test_geometry_under_sanitizers(exe, tmp_path, d, J, M, r, n):
    g0 = np.random.default_rng(M + 10 * d)
    locs = g0.random((n, d))
    locs[:5] = 0.5
    locs[5] = 1.0
    locs[6] = 0.0
    st, res = _geometry(exe, tmp_path, _cfg(d, M, J, r), locs)
    assert st == 0
    info, perm, off, raw, q = res
    og = Geometry(locs, d, M, J, r)
    assert (perm == og.perm).all() and (off == og.offsets).all()
    for a, b in zip(_knots_from(raw, q, og), og.knots):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("Jl,rl,adaptive", [((2, 2, 4, 8), (16, 9, 9, 4), True), ((8, 4, 2), (4, 4, 4), True),
                                            ((16, 16), (4, 9), False)])
def test_mixed_adaptive_geometry_under_sanitizers(exe, tmp_path, Jl, rl, adaptive):
    w = wl.clustered(n=6000, M=len(Jl))
    M = len(Jl)
    pred = np.random.default_rng(4).random((300, 2))
    st, res = _geometry(exe, tmp_path, _cfg(2, M, 4, 4, Jl, rl, adaptive), w.locs, pred=pred)
    assert st == 0
    info, perm, off, raw, q = res
    og = Geometry(w.locs, 2, M, 4, 4, J_levels=Jl, r_levels=rl, adaptive=adaptive)
    assert (perm == og.perm).all() and (off == og.offsets).all()
    for a, b in zip(_knots_from(raw, q, og), og.knots):
        assert np.array_equal(a, b)


def test_explicit_knots_and_refusals_under_sanitizers(exe, tmp_path):
    g0 = np.random.default_rng(3)
    locs = g0.random((100, 2))
    kn = [g0.random((4 ** m, 9, 2)) for m in range(2)]
    st, res = _geometry(exe, tmp_path, _cfg(2, 2, 4, 9), locs, knots=kn)
    assert st == 0
    _, _, _, raw, q = res
    og = Geometry(locs, 2, 2, 4, 9, knots=kn)
    for a, b in zip(_knots_from(raw, q, og), kn):
        assert np.array_equal(a, b)
    bad = locs.copy()
    bad[7] = [np.nan, 0.5]
    assert _geometry(exe, tmp_path, _cfg(2, 2, 4, 9), bad)[0] == _lib.MRA_EINVAL
    assert _geometry(exe, tmp_path, _cfg(2, 2, 3, 9), locs)[0] == _lib.MRA_EINVAL
