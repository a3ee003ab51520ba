"""Benchmark: solid-angle labeling of the four-shell head workload on one GPU.

Workload: four spherical-harmonic perturbed shells (scalp / skull / CSF /
brain, base radii 92 / 86 / 80 / 76 mm, 20,480 triangles each) and the
centroids of a 2 mm Kuhn lattice over [-100, 100]^3 (100^3 cells x 6 =
6,000,000 points), float32 solid angles with the FP64 recheck.  One step
labels every centroid (pair loop, flags, recheck, labels); the centroids are
generated on the GPU and resident in HBM before the timed region.

Prints one JSON line: G point-triangle pairs/s of the FP32+recheck form, the
plain FP64 form on the same workload, the roofline of the dominant kernel and
the FP64 CPU oracle timed on this host's cores over a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 75          # algorithmic FP32 flops of one VOS evaluation (FMA = 2)
FP32_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
FP64_PEAK_TFLOPS = 78.6      # MI355X published FP64 vector peak
COUNTERS_FILE = os.path.join(ROOT, "profiles", "pairloop_f32_c2_hbm_counters.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"],
                    help="c2 (default, the benchmark line); c3 refine-and-relabel, c4 batched, "
                         "c5 precision stress: recheck fraction and oracle mismatches")
    ap.add_argument("--rule", default="centroid", choices=["centroid", "four_nodes"],
                    help="element rule of the c3 refine-and-relabel run")
    ap.add_argument("--conform", action="store_true",
                    help="c3: then build the conforming transition mesh and check it")
    ap.add_argument("--smooth", action="store_true",
                    help="c3: conforming mesh, then Taubin smoothing (implies --conform)")
    ap.add_argument("--cull", action="store_true",
                    help="c3: label with bounding-box culling (pairs/s then counts the skipped "
                         "pairs as well: an effective rate)")
    ap.add_argument("--converge", action="store_true",
                    help="c3: the recursion until the label boundary stops changing "
                         "(finest level = the config's rounds) instead of fixed rounds")
    ap.add_argument("--fp64-round0", action="store_true",
                    help="c3: also time the plain FP64 form on round 0 (the whole lattice)")
    ap.add_argument("--no-c3-leg", action="store_true",
                    help="c2 line: leave out the full c3 refine-and-relabel leg")
    ap.add_argument("--inflate", action="store_true",
                    help="c3: conforming mesh, smoothing, then inflation (implies --smooth)")
    ap.add_argument("--smooth-iters", type=int, default=10,
                    help="iterations per phase of the fixed-count smoothing run")
    ap.add_argument("--c5-lattice-fraction", type=float, default=0.125,
                    help="c5: fraction of the 0.5 mm lattice (a slab along z) to label; "
                         "1 labels all of it")
    ap.add_argument("--c5-slab-fraction", type=float, default=0.0625,
                    help="c5: the lattice is labeled in z-slabs of this fraction of it")
    ap.add_argument("--check-sample", type=int, default=20000,
                    help="c3/c4: points checked against the FP64 oracle")
    ap.add_argument("--c5-check", type=int, default=2000,
                    help="c5: points checked against the FP64 oracle (2.4M triangles each)")
    return ap.parse_args()


def calibrate_copy():
    """A plain device-to-device copy of 1 GiB, three times: reads and writes
    exactly 1 GiB each per launch, the reference for FETCH_SIZE / WRITE_SIZE.
    Also reports the copy's achieved HBM rate (read + write bytes per second)
    as a check of the bandwidth side of the roofline."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    nbytes = src.numel() * 4
    print(json.dumps({"copy_bytes": nbytes, "launches": 4, "ms_per_copy": ms,
                      "hbm_gb_per_s": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)


def source_digest():
    """Hash of the float32 pair-loop sources (kernel and its strip walk)."""
    h = hashlib.sha256()
    for name in ("pairloop.hip", "pairloop_f32.h"):
        h.update(open(os.path.join(ROOT, "paper_2203_10000_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def hbm_traffic(pairloop_launch_pairs):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    try:
        c = json.load(open(COUNTERS_FILE))
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha") != source_digest():
        return None
    return c.get("hbm_bytes_per_launch")


def cpu_baseline(cfg, lat, target_s, rng_seed=7):
    """The FP64 oracle on a bounded random sample of the lattice centroids
    (computed by the oracle itself), all host cores."""
    import numpy as np
    import oracle
    from oracle import kuhn
    rng = np.random.default_rng(rng_seed)
    all_keys = kuhn.level0_keys(lat.cells)
    threads = oracle.host_threads()

    def run(n):
        idx = np.sort(rng.choice(len(all_keys), n, replace=False))
        pts = kuhn.centroids_mm(all_keys[idx], lat.origin, lat.h)
        t0 = time.perf_counter()
        lab = oracle.label(pts, cfg.surfaces, n_threads=threads)
        dt = time.perf_counter() - t0
        return idx, lab, dt

    n = 512
    _, _, dt = run(n)
    n = int(min(len(all_keys), max(n, n * target_s / max(dt, 1e-3))))
    idx, lab, dt = run(n)
    pairs = n * cfg.n_tri
    return {"value": pairs / dt / 1e9, "unit": "G pairs/s", "cores": threads, "kind": "oracle",
            "sample": "%d lattice centroids drawn uniformly from the 6,000,000 (x %d triangles "
                      "= %.3g pairs), FP64 VOS with exact-sign guard, %.1f s" % (n, cfg.n_tri,
                                                                                pairs, dt),
            "cpu_model": cpu_model()}, idx, lab


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def progress(msg):
    """Phase line on stderr (long measurement runs print as they go)."""
    print("[%s] %s" % (time.strftime("%H:%M:%S"), msg), file=sys.stderr, flush=True)


def _oracle_check(pts_np, surfaces, gpu_labels_np, n, rng, near_mask=None):
    """Labels of a sample (uniform + near-surface) against the FP64 oracle."""
    import numpy as np
    import oracle
    progress("oracle check of %d (+%d near) points" % (n, n if near_mask is not None else 0))
    idx = rng.choice(pts_np.shape[1], min(n, pts_np.shape[1]), replace=False)
    if near_mask is not None and near_mask.any():
        near = np.nonzero(near_mask)[0]
        idx = np.unique(np.concatenate([idx, rng.choice(near, min(n, len(near)), replace=False)]))
    threads = oracle.host_threads()
    t0 = time.perf_counter()
    want = oracle.label(np.ascontiguousarray(pts_np[:, idx]), surfaces, n_threads=threads)
    dt = time.perf_counter() - t0
    n_tri = sum(len(s.f) for s in surfaces)
    _ORACLE_RATE.update({"value": len(idx) * n_tri / max(dt, 1e-9) / 1e9, "unit": "G pairs/s",
                         "cores": threads, "kind": "oracle",
                         "sample": "%d points x %d triangles, %.1f s" % (len(idx), n_tri, dt)})
    return int((gpu_labels_np[idx] != want).sum()), int(len(idx))


# The oracle's rate on the last label check (reported beside the c3-c5 results).
_ORACLE_RATE = {}

RADIAL_METHOD = ("exact radial point-in-polyhedron test (oracle): the cone from the surface's "
                 "centre that holds the point, then the exact orient3d side")


def _radial_result(kind, checked, mism, bad, dt, threads):
    return {"method": RADIAL_METHOD, "points": kind, "checked": int(checked),
            "mismatches": int(mism), "first_mismatches": [int(b) for b in bad[:8]],
            "s": round(dt, 2), "cores": threads}


def exact_check_lattice(surfaces, lat, labels_np, first=0, what="every lattice centroid"):
    """Every label of lattice points first .. first + len - 1 against the
    radial test (the oracle forms the centroids itself)."""
    import oracle
    threads = oracle.host_threads()
    t0 = time.perf_counter()
    rs = oracle.RadialSet(surfaces)
    mism, bad = rs.check_lattice(lat, labels_np, first=first, n_threads=threads)
    return _radial_result(what, len(labels_np), mism, bad, time.perf_counter() - t0, threads)


def exact_check_keys(surfaces, origin, h, keys_np, labels_np, rule):
    """Every leaf label (centroid or four-node rule) against the radial test."""
    import oracle
    threads = oracle.host_threads()
    t0 = time.perf_counter()
    rs = oracle.RadialSet(surfaces)
    mism, bad = rs.check_keys(origin, h, keys_np, labels_np, rule=rule, n_threads=threads)
    what = "every leaf (%s rule)" % ("centroid" if rule == "centroid" else "four-node")
    return _radial_result(what, len(labels_np), mism, bad, time.perf_counter() - t0, threads)


def exact_check_points(surfaces, pts_np, labels_np, what="every point"):
    """Every label of explicit points [3, N] against the radial test."""
    import numpy as np
    import oracle
    threads = oracle.host_threads()
    t0 = time.perf_counter()
    want = oracle.RadialSet(surfaces).label(pts_np, n_threads=threads)
    bad = np.nonzero(want != labels_np)[0]
    return _radial_result(what, len(labels_np), len(bad), bad, time.perf_counter() - t0, threads)


def _oracle_check_nodes(keys, lat, surfaces, gpu_labels_np, n, rng, near_mask=None):
    """Four-node rule: a sample of leaves, each labeled by the oracle from the
    enclosure masks of its four nodes."""
    import numpy as np
    import oracle
    from oracle import kuhn
    progress("oracle check of %d (+%d near) leaves, four-node rule" %
             (n, n if near_mask is not None else 0))
    idx = rng.choice(len(keys), min(n, len(keys)), replace=False)
    if near_mask is not None and near_mask.any():
        near = np.nonzero(near_mask)[0]
        idx = np.unique(np.concatenate([idx, rng.choice(near, min(n, len(near)), replace=False)]))
    v = kuhn.vertices_units(keys[idx]).reshape(-1, 3)
    pts = kuhn.nodes_mm(v, lat.origin, lat.h)
    threads = oracle.host_threads()
    t0 = time.perf_counter()
    m = oracle.enclosure(pts, surfaces, n_threads=threads).reshape(-1, 4)
    dt = time.perf_counter() - t0
    want = oracle.mask_label(m[:, 0] & m[:, 1] & m[:, 2] & m[:, 3], surfaces)
    n_tri = sum(len(s.f) for s in surfaces)
    _ORACLE_RATE.update({"value": pts.shape[1] * n_tri / max(dt, 1e-9) / 1e9, "unit": "G pairs/s",
                         "cores": threads, "kind": "oracle",
                         "sample": "%d nodes x %d triangles, %.1f s" % (pts.shape[1], n_tri, dt)})
    return int((gpu_labels_np[idx] != want).sum()), int(len(idx))


def _conform_c3(mesh, lat, rng, n_sample=200000):
    """Conforming transition mesh of the refined c3 leaves, timed, with checks
    that hold at any size: positive volumes that sum exactly to the box, and
    no node at an edge midpoint of a sampled tetrahedron."""
    import numpy as np
    import torch
    progress("c3: conforming transition mesh")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = mesh.conform()
    wall = time.perf_counter() - t0
    e = mesh.export_conforming()
    keys = e["node_keys"]
    m = 0x1FFFFF
    pts = torch.stack([(keys >> 42) & m, (keys >> 21) & m, keys & m], 1)     # [n, 3] int64
    tets = e["tets"].long()
    v6 = torch.zeros(len(tets), dtype=torch.int64, device=tets.device)
    for lo in range(0, len(tets), 1 << 24):
        p = pts[tets[lo:lo + (1 << 24)]]
        a, b, c = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
        v6[lo:lo + len(p)] = (a[:, 0] * (b[:, 1] * c[:, 2] - b[:, 2] * c[:, 1])
                              - a[:, 1] * (b[:, 0] * c[:, 2] - b[:, 2] * c[:, 0])
                              + a[:, 2] * (b[:, 0] * c[:, 1] - b[:, 1] * c[:, 0]))
    box6 = 6 * int(np.prod(np.array(lat.cells, dtype=np.int64) * 8))
    idx = torch.from_numpy(rng.choice(len(tets), min(n_sample, len(tets)), replace=False)).to(tets.device)
    p = pts[tets[idx]]
    hanging = 0
    for i, j in [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]:
        s2 = p[:, i] + p[:, j]
        ok = (s2 % 2 == 0).all(1)
        mk = ((s2[:, 0] // 2) << 42) | ((s2[:, 1] // 2) << 21) | (s2[:, 2] // 2)
        pos = torch.searchsorted(keys, mk).clamp(max=len(keys) - 1)
        hanging += int((ok & (keys[pos] == mk)).sum())
    torch.cuda.synchronize()
    res = dict(info)
    res.update({"wall_s": wall, "leaves_per_s": info["n_leaves"] / wall,
                "volumes_positive": bool((v6 > 0).all()), "volume_sum_exact": int(v6.sum()) == box6,
                "hanging_nodes_in_sample": hanging, "sample_tets": int(len(idx))})
    del e, pts, tets, v6
    return res


def _smooth_c3(mesh, iters):
    """Taubin smoothing of the c3 conforming mesh: once with the paper's
    parameters (edge graph built on this call), then `iters` iterations per
    phase with the stopping rule off, timed per half step.  Bytes per half
    step: every array read or written once (node list 4, row pointer 8,
    columns 4 per entry, positions 16 per node read, 16 per node written)."""
    import torch
    progress("c3: Taubin smoothing")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    paper = mesh.smooth()
    wall = time.perf_counter() - t0
    fixed = mesh.smooth(xi_surface=-1.0, xi_volume=-1.0, max_iter_surface=iters,
                        max_iter_volume=iters)
    n_nodes = mesh.conform_info["n_nodes"]
    out = {"paper_params": paper, "paper_params_wall_s": wall, "fixed_iterations": fixed}
    for ph in ("surface", "volume"):
        n = fixed["n_%s_nodes" % ph]
        ent = fixed["n_entries_%s" % ph]
        halves = 2 * fixed["iters_%s" % ph]
        if not halves:
            continue
        ms = fixed["ms_%s" % ph] / halves
        nbytes = 4 * n + 8 * n + 4 * ent + 16 * min(n_nodes, n + ent) + 16 * n
        out["%s_half_step" % ph] = {"ms": ms, "nodes": n, "entries": ent, "bytes": nbytes,
                                    "gb_per_s": nbytes / (ms * 1e-3) / 1e9,
                                    "frac_of_8tb": nbytes / (ms * 1e-3) / 8e12}
    return out


def _inflate_c3(mesh, ss):
    """Inflation of the smoothed c3 mesh with zeta = 0.05 (timed by the
    library's events: triangle binning, then the move)."""
    progress("c3: inflation")
    first = mesh.inflate(ss, 0.05)
    again = mesh.inflate(ss, 0.05)
    ms = again["ms_inflate"]
    return {"first": first, "second": again,
            "triangle_tests_per_s": again["n_triangle_tests"] / (ms * 1e-3),
            "edges_per_s": again["n_edges_tested"] / (ms * 1e-3)}


def run_c3(args, fp64_sample=True):
    """c3: 20 compartments (4 x 81,920 + 16 x 5,120 triangles), 1 mm lattice
    (48M centroids), two refine-and-relabel rounds in FP32 + recheck.  Every
    leaf label is checked by the exact radial test; with `fp64_sample` a
    sample is also labeled by the FP64 oracle (its CPU rate)."""
    import numpy as np
    import torch
    import paper_2203_10000_amd as sal
    import synth
    progress("c3: generating surfaces")
    cfg = synth.config_c3()
    lat = cfg.lattice
    progress("c3: labeling and refining (%s rule)" % args.rule)
    ctx = sal.Context(0)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    converged = None
    if getattr(args, "converge", False):
        st, converged = mesh.refine_converge(ss, cfg.rounds, max_steps=32, precision="fp32",
                                             rule=args.rule, cull=args.cull)
    else:
        st = mesh.refine_relabel(ss, cfg.rounds, precision="fp32", rule=args.rule, cull=args.cull)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pairs = sum(r["n_pairs"] for r in st)
    ms_label = sum(r["ms_label"] for r in st)
    n_leaves, lv = mesh.size()
    e = mesh.export(keys=True, labels=True, centroids=fp64_sample and args.rule == "centroid")
    lab = e["labels"].cpu().numpy()
    keys = e["keys"].cpu().numpy().view(np.uint64)
    cen = e["centroids"].cpu().numpy() if e["centroids"] is not None else None
    del e
    progress("c3: exact radial check of all %d leaves" % n_leaves)
    exact = exact_check_keys(cfg.surfaces, lat.origin, lat.h, keys, lab, args.rule)
    mism = checked = None
    if fp64_sample:
        rng = np.random.default_rng(33)
        if args.rule == "four_nodes":
            import oracle
            r = np.linalg.norm(oracle.leaf_points(lat.origin, lat.h, keys).astype(np.float64), axis=0)
        else:
            r = np.linalg.norm(cen.astype(np.float64), axis=0)
        near = np.min(np.abs(r[:, None] - np.array([92, 86, 80, 76.0])), axis=1) < 4.0
        if args.rule == "four_nodes":
            mism, checked = _oracle_check_nodes(keys, lat, cfg.surfaces, lab, args.check_sample,
                                                rng, near)
        else:
            mism, checked = _oracle_check(cen, cfg.surfaces, lab, args.check_sample, rng, near)
    out = {"workload": "c3", "rule": args.rule, "cull_bounds": bool(args.cull),
           "recursion": "converging" if converged is not None else "fixed rounds",
           "converged": converged,
           "triangles": cfg.n_tri, "rounds": st, "leaves": n_leaves, "max_level": lv,
           "pairs": pairs, "wall_s": wall, "g_pairs_per_s": pairs / wall / 1e9,
           "pairloop_ms": ms_label,
           "roofline": pairloop_roofline(pairs, ms_label, "k_pairloop_f32 (all rounds)"),
           "leaf_count_identity": n_leaves == lat.n_points + 7 * sum(x["n_boundary"] for x in st),
           "exact_label_check": exact}
    if fp64_sample:
        out.update({"oracle_sample_mismatches": mism, "oracle_sample": checked,
                    "oracle_rate": dict(_ORACLE_RATE)})
    if getattr(args, "fp64_round0", False):
        out["fp64_round0"] = _c3_fp64_round0(ctx, ss, cfg, lat, args.rule)
    post = args.conform or args.smooth or args.inflate
    if post:
        rng = np.random.default_rng(34)
        out["conform"] = _conform_c3(mesh, lat, rng)
        out["smooth"] = _smooth_c3(mesh, args.smooth_iters) if (args.smooth or args.inflate) else None
        out["inflate"] = _inflate_c3(mesh, ss) if args.inflate else None
    return out


def _c3_fp64_round0(ctx, ss, cfg, lat, rule):
    """The plain FP64 form on c3's round 0 (the whole 1 mm lattice), each
    label checked by the radial test."""
    import numpy as np
    import torch
    import paper_2203_10000_amd as sal
    progress("c3: plain FP64 form on round 0 (%s rule)" % rule)
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = mesh.refine_relabel(ss, 0, precision="fp64", rule=rule)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e = mesh.export(keys=rule != "centroid", labels=True, centroids=False)
    lab = e["labels"].cpu().numpy()
    if rule == "centroid":
        exact = exact_check_lattice(cfg.surfaces, lat, lab)
    else:
        exact = exact_check_keys(cfg.surfaces, lat.origin, lat.h,
                                 e["keys"].cpu().numpy().view(np.uint64), lab, rule)
    pairs = st[0]["n_pairs"]
    return {"pairs": pairs, "wall_s": wall, "g_pairs_per_s": pairs / wall / 1e9,
            "pairloop_ms": st[0]["ms_label"],
            "roofline": pairloop_roofline(pairs, st[0]["ms_label"], "k_pairloop_f64", fp64=True),
            "exact_label_check": exact}


def pairloop_roofline(pairs, ms, kernel, fp64=False):
    """ALU roofline of a pair-loop launch (75 algorithmic flops per pair)."""
    peak = FP64_PEAK_TFLOPS if fp64 else FP32_PEAK_TFLOPS
    achieved = FLOPS_PER_PAIR * pairs / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 2), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "flops_per_pair": FLOPS_PER_PAIR,
            "kernel_ms": round(ms, 3), "pairs": pairs}


def run_c4(args):
    """c4: 64 instances, batched persistent launch (eager and hipGraph replay)
    against 64 per-instance launches, in FP32 + recheck and in the plain FP64
    form; every label checked by the radial test."""
    import numpy as np
    import torch
    import paper_2203_10000_amd as sal
    import synth
    progress("c4: generating 64 instances")
    insts = synth.config_c4()
    ctx = sal.Context(0)
    progress("c4: timing")
    dev = []
    pairs = 0
    for surfs, pts in insts:
        ss = sal.SurfaceSet(ctx, surfs)
        p = torch.from_numpy(pts).to("cuda:0")
        dev.append((ss, p, torch.empty(pts.shape[1], dtype=torch.int32, device="cuda:0")))
        pairs += pts.shape[1] * sum(s.n_tri for s in surfs)
    out = {"workload": "c4", "instances": len(insts), "pairs": pairs,
           "points": int(sum(p.shape[1] for _, p in insts))}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    per = [torch.empty_like(l) for _, _, l in dev]

    def per_instance(prec):
        for (ss, p, _), l in zip(dev, per):
            sal.label_points(ctx, ss, p, out=l, precision=prec)

    t_per = timed(lambda: per_instance("fp32"), 2)
    t_batch = timed(lambda: sal.label_batch(ctx, dev), 2)
    t_graph = timed(lambda: sal.label_batch(ctx, dev, use_graph=True), 3)
    same = all(torch.equal(a, l) for a, (_, _, l) in zip(per, dev))
    progress("c4: exact radial check of every label")
    exact = _c4_exact(insts, [l.cpu().numpy() for _, _, l in dev])
    rng = np.random.default_rng(44)
    mism = checked = 0
    for (surfs, pts), (_, _, l) in list(zip(insts, dev))[:16]:
        m, c = _oracle_check(pts, surfs, l.cpu().numpy(), args.check_sample // 16, rng)
        mism += m
        checked += c
    out.update({"per_instance": {"s": t_per, "g_pairs_per_s": pairs / t_per / 1e9},
                "batched": {"s": t_batch, "g_pairs_per_s": pairs / t_batch / 1e9},
                "batched_graph": {"s": t_graph, "g_pairs_per_s": pairs / t_graph / 1e9},
                "batched_equals_per_instance": bool(same),
                "exact_label_check": exact,
                "oracle_sample_mismatches": mism, "oracle_sample": checked,
                "oracle_rate": dict(_ORACLE_RATE)})
    if args.fp64_steps > 0:
        progress("c4: plain FP64 form, per instance and batched")
        t64_per = timed(lambda: per_instance("fp64"), 1)
        t64_batch = timed(lambda: sal.label_batch(ctx, dev, precision="fp64"), 1)
        t64_graph = timed(lambda: sal.label_batch(ctx, dev, precision="fp64", use_graph=True), 1)
        same64 = all(torch.equal(a, l) for a, (_, _, l) in zip(per, dev))
        exact64 = _c4_exact(insts, [l.cpu().numpy() for _, _, l in dev])
        out["fp64_form"] = {"per_instance": {"s": t64_per, "g_pairs_per_s": pairs / t64_per / 1e9},
                            "batched": {"s": t64_batch, "g_pairs_per_s": pairs / t64_batch / 1e9},
                            "batched_graph": {"s": t64_graph,
                                              "g_pairs_per_s": pairs / t64_graph / 1e9},
                            "batched_equals_per_instance": bool(same64),
                            "exact_label_check": exact64}
    return out


def _c4_exact(insts, labels):
    """Radial check of every label of every instance."""
    tot = {"checked": 0, "mismatches": 0, "s": 0.0}
    for (surfs, pts), lab in zip(insts, labels):
        r = exact_check_points(surfs, pts, lab)
        for k in tot:
            tot[k] += r[k]
        cores = r["cores"]
    tot.update({"method": RADIAL_METHOD, "points": "every point of the 64 instances",
                "cores": cores, "s": round(tot["s"], 2)})
    return tot


def run_c5(args):
    """c5: 8 x 297,680-triangle compartments; 2e7 points offset U[-0.5, 0.5] mm
    along face normals, and the 0.5 mm lattice over the outer shell's box
    (z-slabs of --c5-lattice-fraction of it, labeled one after the other);
    recheck fractions, rates and a radial check of every label."""
    import numpy as np
    import torch
    import oracle
    import paper_2203_10000_amd as sal
    import synth
    progress("c5: generating surfaces and points")
    cfg = synth.config_c5()
    lat = cfg.lattice
    ctx = sal.Context(0)
    progress("c5: near-surface points")
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    out = {"workload": "c5", "triangles": cfg.n_tri, "lattice_cells": lat.cells,
           "lattice_points": lat.n_points}
    near = torch.from_numpy(cfg.points).to("cuda:0")
    torch.cuda.synchronize()
    t = time.perf_counter()
    lab, _, st = sal.label_points(ctx, ss, near, stats=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    lab_np = lab.cpu().numpy()
    progress("c5: exact radial check of the %d near-surface labels" % len(lab_np))
    exact = exact_check_points(cfg.surfaces, cfg.points, lab_np, "every near-surface point")
    rng = np.random.default_rng(55)
    mism, checked = _oracle_check(cfg.points, cfg.surfaces, lab_np, args.c5_check, rng)
    out["near_surface"] = {"points": int(near.shape[1]), "pairs": st["n_pairs"], "wall_s": wall,
                           "g_pairs_per_s": st["n_pairs"] / wall / 1e9,
                           "roofline": pairloop_roofline(st["n_pairs"], st["ms_pairloop"],
                                                         "k_pairloop_f32"),
                           "recheck_points": st["n_recheck_points"],
                           "recheck_pairs": st["n_recheck_pairs"],
                           "band_flags": st["n_band_flags"], "cond_flags": st["n_cond_flags"],
                           "exact_fallbacks": st["n_exact_fallbacks"],
                           "ms_pairloop": st["ms_pairloop"], "ms_recheck": st["ms_recheck"],
                           "exact_label_check": exact,
                           "oracle_sample_mismatches": mism, "oracle_sample": checked,
                           "oracle_rate": dict(_ORACLE_RATE)}
    del near, lab, lab_np
    # the lattice, slab by slab along z (each slab a lattice of its own,
    # origin shifted by whole cells: every coordinate stays on the same grid)
    nz = max(1, int(round(lat.cells[2] * args.c5_lattice_fraction)))
    tot = {"points": 0, "pairs": 0, "wall_s": 0.0, "ms_pairloop": 0.0, "ms_recheck": 0.0,
           "recheck_pairs": 0, "band_flags": 0, "cond_flags": 0, "exact_fallbacks": 0,
           "recheck_points": 0, "checked": 0, "mismatches": 0, "check_s": 0.0}
    radial = None
    z0 = 0 if args.c5_lattice_fraction >= 1.0 else (lat.cells[2] - nz) // 2
    z_end = lat.cells[2] if args.c5_lattice_fraction >= 1.0 else z0 + nz
    slab_nz = max(1, int(round(lat.cells[2] * args.c5_slab_fraction)))
    lab_buf = torch.empty(0, dtype=torch.int32, device="cuda:0")
    for za in range(z0, z_end, slab_nz):
        dz = min(slab_nz, z_end - za)
        slab = synth.Lattice(origin=(lat.origin[0], lat.origin[1], lat.origin[2] + lat.h * za),
                             h=lat.h, cells=(lat.cells[0], lat.cells[1], dz))
        mesh = sal.TetMesh(ctx, slab.origin, slab.h, slab.cells)
        cen = mesh.export(keys=False, labels=False, centroids=True)["centroids"]
        if lab_buf.numel() < slab.n_points:
            lab_buf = torch.empty(slab.n_points, dtype=torch.int32, device="cuda:0")
        lab = lab_buf[:slab.n_points]
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, st = sal.label_points(ctx, ss, cen, stats=True, out=lab)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        lab_np = lab.cpu().numpy()
        del cen, mesh
        if radial is None:
            radial = oracle.RadialSet(cfg.surfaces)
        t = time.perf_counter()
        m, bad = radial.check_lattice(slab, lab_np, n_threads=oracle.host_threads())
        tot["check_s"] += time.perf_counter() - t
        tot["checked"] += len(lab_np)
        tot["mismatches"] += m
        tot["points"] += slab.n_points
        tot["pairs"] += st["n_pairs"]
        tot["wall_s"] += wall
        for k in ("ms_pairloop", "ms_recheck"):
            tot[k] += st[k]
        for k in ("recheck_pairs", "band_flags", "cond_flags", "exact_fallbacks",
                  "recheck_points"):
            tot[k] += st["n_" + k]
        progress("c5: lattice z %d..%d of %d: %.1f s, %.0f G pairs/s, %d rechecked pairs, "
                 "%d mismatches (exact check)" % (za, za + dz, lat.cells[2], wall,
                                                  st["n_pairs"] / wall / 1e9,
                                                  st["n_recheck_pairs"], m))
    tot["g_pairs_per_s"] = tot["pairs"] / tot["wall_s"] / 1e9
    tot["roofline"] = pairloop_roofline(tot["pairs"], tot["ms_pairloop"], "k_pairloop_f32")
    tot["z_cells"] = [z0, z_end]
    tot["exact_label_check"] = {"method": RADIAL_METHOD, "checked": tot.pop("checked"),
                                "mismatches": tot.pop("mismatches"),
                                "s": round(tot.pop("check_s"), 2)}
    out["lattice"] = tot
    return out


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(labeling would shard by points, one slab of lattice cells per GPU).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2203_10000_amd as sal
    import synth

    if args.workload != "c2":
        torch.cuda.set_device(0)
        fn = {"c3": run_c3, "c4": run_c4, "c5": run_c5}[args.workload]
        print(json.dumps(fn(args), default=float), flush=True)
        return

    cfg = synth.config_c2()
    lat = cfg.lattice
    n_points = lat.n_points
    pairs = n_points * cfg.n_tri

    torch.cuda.set_device(0)
    ctx = sal.Context(0)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    exp = mesh.export(keys=True, labels=False, centroids=True)     # lattice centroids on the GPU
    cen = exp["centroids"]
    keys_dev = exp["keys"]
    labels = torch.empty(n_points, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()

    def step(precision):
        _, _, st = sal.label_points(ctx, ss, cen, precision=precision, stats=True, out=labels)
        return st

    for _ in range(args.warmup):
        step("fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kstats = []
    for _ in range(args.steps):
        kstats.append(step("fp32"))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = pairs * args.steps / wall / 1e9
    ms_pairloop = float(np.mean([s["ms_pairloop"] for s in kstats]))
    ms_recheck = float(np.mean([s["ms_recheck"] for s in kstats]))
    recheck_pairs = kstats[-1]["n_recheck_pairs"]
    gpu_labels = labels.cpu().numpy()
    gpu_keys = keys_dev.cpu().numpy().view(np.uint64)

    progress("c2: exact radial check of all %d labels" % n_points)
    exact = exact_check_lattice(cfg.surfaces, lat, gpu_labels)

    fp64 = None
    if args.fp64_steps > 0:
        lab64 = torch.empty_like(labels)
        for _ in range(1):                          # untimed: the tuner's trials run here
            sal.label_points(ctx, ss, cen, precision="fp64", out=lab64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms64 = []
        for _ in range(args.fp64_steps):
            _, _, st64 = sal.label_points(ctx, ss, cen, precision="fp64", out=lab64, stats=True)
            ms64.append(st64["ms_pairloop"])
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t1
        fp64 = {"value": pairs * args.fp64_steps / w64 / 1e9, "unit": "G pairs/s",
                "ms_per_step": 1e3 * w64 / args.fp64_steps, "steps": args.fp64_steps,
                "labels_equal_fp32_form": bool(torch.equal(lab64, labels)),
                "roofline": pairloop_roofline(pairs, float(np.mean(ms64)), "k_pairloop_f64",
                                              fp64=True)}

    achieved = FLOPS_PER_PAIR * pairs / (ms_pairloop * 1e-3) / 1e12
    traffic = hbm_traffic(pairs)
    kernel = "k_pairloop_f32<%d, false>" % kstats[-1]["points_per_lane"]
    roofline = {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 2),
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": traffic, "flops_per_pair": FLOPS_PER_PAIR,
                "kernel_ms": round(ms_pairloop, 3), "pairs_per_launch": pairs}

    cpu = None
    if not args.no_cpu_baseline:
        cpu, oidx, olab = cpu_baseline(cfg, lat, args.cpu_seconds)
        # both sides number the lattice ((k ny + j) nx + i) 6 + q
        from oracle import kuhn
        assert np.array_equal(gpu_keys[oidx], kuhn.level0_keys(lat.cells)[oidx])
        cpu["sample_label_mismatches_vs_gpu"] = int((gpu_labels[oidx] != olab).sum())

    c3 = None
    if not args.no_c3_leg:
        # the largest single-GPU workload, once: refine-and-relabel, every leaf checked
        del exp, cen, keys_dev, labels
        torch.cuda.empty_cache()
        args.rule, args.cull = "centroid", False
        c3 = run_c3(args, fp64_sample=False)
        c3 = {k: c3[k] for k in ("workload", "rule", "triangles", "leaves", "max_level", "pairs",
                                 "wall_s", "g_pairs_per_s", "pairloop_ms", "roofline",
                                 "leaf_count_identity", "exact_label_check")}
        c3["config"] = ("20 compartments (4 SH shells x 81,920 + 16 ellipsoids x 5,120 "
                        "triangles), 1 mm Kuhn lattice (48,000,000 centroids), round 0 + 2 "
                        "refine-and-relabel rounds, FP32 + FP64 recheck")

    out = {
        "metric": "G point-triangle solid-angle pairs/s (FP32+recheck vs FP64) and % FP32 VALU peak",
        "value": round(value, 2),
        "unit": "G pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "four SH-perturbed shells (92/86/80/76 mm, 4 x 20,480 triangles), "
                               "2 mm Kuhn lattice over [-100,100]^3 (6,000,000 centroids), "
                               "FP32 + FP64 recheck (band 1e-3)",
                   "points": n_points, "triangles": cfg.n_tri, "pairs_per_step": pairs},
        "fp64_form": fp64,
        "recheck": {"pairs": recheck_pairs, "fraction_of_points": recheck_pairs / n_points,
                    "ms_recheck": round(ms_recheck, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "exact_label_check": exact,
        "c3_refine_relabel": c3,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
