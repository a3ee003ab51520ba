"""The oracle (sal_oracle.c, radial.c) and the host-only parts of libsal
(surface validation and strips, the tuner's cache file) built with gcc under
AddressSanitizer and UndefinedBehaviorSanitizer, run on seeded inputs; their
results must equal the normal builds' (liboracle.so, libsal.so), so the
sanitized run checks the code paths the tests rely on.  CPU only."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle import kuhn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.fixture(scope="module")
def bins(tmp_path_factory):
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("san")
    od, hd = str(d / "oracle_driver"), str(d / "host_driver")
    _build(["gcc"] + SAN + ["-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"),
                            os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                            os.path.join(ROOT, "oracle", "sal_oracle.c"),
                            os.path.join(ROOT, "oracle", "radial.c"), "-lpthread", "-lm", "-o", od])
    csrc = os.path.join(ROOT, "paper_2203_10000_amd", "csrc")
    _build(["g++", "-std=c++17"] + SAN + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                                          "-I", os.path.join(ROOT, "include"), "-I", csrc,
                                          os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                                          os.path.join(csrc, "surface_host.cpp"),
                                          os.path.join(csrc, "tune_cache.cpp"), "-o", hd])
    return d, od, hd


def _run(args):
    r = subprocess.run(args, capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, "sanitized run failed:\n" + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_oracle_under_sanitizers_matches_the_normal_build(bins):
    d, od, _ = bins
    cfg = synth.config_small("head", cells=6, subdiv=2)
    surfs = cfg.surfaces
    rng = np.random.default_rng(5)
    pts = np.concatenate([synth.uniform_box(rng, 3000, -100, 100),
                          synth.near_surface_points(rng, surfs, 2000, 0.5),
                          synth.face_centroids_on_surface(surfs[0], 64)], 1).astype(np.float32)
    lat = cfg.lattice
    k0 = kuhn.level0_keys(lat.cells)
    keys = np.concatenate([k0[::7], kuhn.children(k0[::53], lat.cells).reshape(-1)])
    blob = [struct.pack("<i", len(surfs))]
    for s in surfs:
        blob += [struct.pack("<qqi", len(s.v), len(s.f), s.label),
                 np.asarray(s.center, np.float32).tobytes(), s.v.astype(np.float32).tobytes(),
                 s.f.astype(np.int32).tobytes()]
    blob += [struct.pack("<q", pts.shape[1]), pts[0].tobytes(), pts[1].tobytes(), pts[2].tobytes(),
             np.asarray(lat.origin, np.float64).tobytes(), struct.pack("<d", lat.h),
             np.asarray(lat.cells, np.int64).tobytes(), struct.pack("<q", len(keys)),
             keys.astype(np.uint64).tobytes()]
    inp, outp = str(d / "oracle_in.bin"), str(d / "oracle_out.bin")
    with open(inp, "wb") as f:
        f.write(b"".join(blob))
    _run([od, inp, outp])
    raw = open(outp, "rb").read()
    n, ns, nk = pts.shape[1], len(surfs), len(keys)
    off = 0

    def take(dtype, count):
        nonlocal off
        a = np.frombuffer(raw, dtype=dtype, count=count, offset=off)
        off += a.nbytes
        return a

    lab, w = oracle.label(pts, surfs, want_w=True, n_threads=2)
    assert np.array_equal(take(np.int32, n), lab)
    assert np.array_equal(take(np.float64, ns * n), w.reshape(-1))
    assert np.array_equal(take(np.uint64, n), oracle.enclosure(pts, surfs, n_threads=2))
    rs = oracle.RadialSet(surfs)
    rl, rm = rs.label(pts, n_threads=2, want_masks=True)
    assert np.array_equal(take(np.int32, n), rl)
    assert np.array_equal(take(np.uint64, n), rm)
    zeros = np.zeros(lat.n_points, np.int32)
    mism = take(np.int64, 3)
    assert mism[0] == rs.check_lattice(lat, zeros, n_threads=2)[0]
    assert mism[1] == rs.check_keys(lat.origin, lat.h, keys, zeros[:nk], n_threads=2)[0]
    assert mism[2] == rs.check_keys(lat.origin, lat.h, keys, zeros[:nk], rule="four_nodes",
                                    n_threads=2)[0]
    assert mism[0] > 0 and mism[1] > 0
    assert np.array_equal(take(np.float32, 3 * nk).reshape(nk, 3).T,
                          oracle.leaf_points(lat.origin, lat.h, keys))
    assert np.array_equal(take(np.float32, 12 * nk).reshape(nk, 4, 3),
                          oracle.leaf_points(lat.origin, lat.h, keys, rule="four_nodes"))
    w0, on0 = oracle.winding(pts, surfs[0].v, surfs[0].f, n_threads=2)
    assert np.array_equal(take(np.float64, n), w0)
    assert np.array_equal(take(np.uint8, n).astype(bool), on0)
    assert on0.sum() >= 64
    assert np.array_equal(take(np.uint8, n), oracle.radial_inside(pts, surfs[0], n_threads=2))
    assert off == len(raw)


def _cases():
    """(flags, surfaces as (v, f, label), expected status)."""
    v, f = synth.icosphere(2)
    v = (v * 50).astype(np.float32)
    f = f.astype(np.int32)
    rev = f[:, [0, 2, 1]].copy()
    nan = v.copy()
    nan[3, 1] = np.nan
    oob = f.copy()
    oob[0, 0] = len(v) + 5
    rep = f.copy()
    rep[0, 1] = rep[0, 0]
    dup = np.concatenate([f, f[:1]])
    flat = v.copy()
    a, b, c = f[0]
    flat[c] = flat[a]                                  # triangle 0 has zero area
    head = synth.config_small("head", subdiv=2).surfaces
    return [
        (0, [(v, f, 1)], 0),
        (0, [(s.v, s.f, s.label) for s in head], 0),
        (0, [(v, f[1:], 1)], 2),                      # open
        (0, [(v, rev, 1)], 3),                        # inward
        (1, [(v, rev, 1)], 0),                        # inward, auto-oriented
        (0, [(nan, f, 1)], 1),                        # non-finite vertex
        (0, [(v, oob, 1)], 1),                        # index out of range
        (0, [(v, rep, 1)], 1),                        # triangle repeats a vertex
        (0, [(v, dup, 1)], 2),                        # a directed edge twice
        (0, [(flat, f, 1)], 1),                       # zero-area triangle
        (0, [(v, f, 0)], 1),                          # label must be > 0
        (0, [(v, f, 1)] * 65, 1),                     # too many surfaces
        (0, [(v[:2], f[:2], 1)], 1),                  # too small
    ]


def test_host_library_parts_under_sanitizers(bins):
    import paper_2203_10000_amd as sal
    d, _, hd = bins
    cases = _cases()
    blob = [struct.pack("<i", len(cases))]
    for flags, surfs, _ in cases:
        blob.append(struct.pack("<ii", flags, len(surfs)))
        for v, f, label in surfs:
            blob += [struct.pack("<qqi", len(v), len(f), label), np.asarray(v, np.float32).tobytes(),
                     np.asarray(f, np.int32).tobytes()]
    inp, outp = str(d / "host_in.bin"), str(d / "host_out.bin")
    with open(inp, "wb") as fh:
        fh.write(b"".join(blob))
    tune_in, tune_out = str(d / "tune_in.txt"), str(d / "tune_out.txt")
    with open(tune_in, "w") as fh:
        fh.write("gfx950:sramecc+:xnack- 0 1 16 19 0 0 1 8\n"
                 "gfx950:sramecc+:xnack- 0 0 16 19 1 0 1 4\n"
                 "gfx950:sramecc+:xnack- 0 0 12 14 0 0 2 4\n"
                 + "g" * 300 + " 0 0 1 1 0 0 1 1\n"
                 "gfx950 0 0 9 9 0 0 4 8\n")
    out = _run([hd, inp, outp, tune_in, tune_out])
    assert out.split() == ["tune", "entries", "3", "3"]      # reading stops at the bad line
    raw = open(outp, "rb").read()
    rec = struct.Struct("<iiqqq")
    assert len(raw) == rec.size * len(cases)
    for i, (flags, surfs, want) in enumerate(cases):
        st, ns, nt, nstrip, nbytes = rec.unpack_from(raw, i * rec.size)
        assert st == want, (i, st, want)
        if want == 0:
            info = sal.surface_set_check(surfs, auto_orient=bool(flags))
            assert (ns, nt, nstrip, nbytes) == (info["n_surfaces"], info["n_triangles"],
                                                info["n_strips"], info["device_bytes"])
            assert nt == sum(len(f) for _, f, _ in surfs)
        else:
            with pytest.raises(sal.SalError) as e:
                sal.surface_set_check(surfs, auto_orient=bool(flags))
            assert e.value.status == want
