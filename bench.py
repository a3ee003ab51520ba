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
    return ap.parse_args()


def calibrate_copy():
    """A plain device-to-device copy of 1 GiB, three times: reads and writes
    exactly 1 GiB each per launch, the reference for FETCH_SIZE / WRITE_SIZE."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 4, "launches": 3}), flush=True)


def source_digest():
    p = os.path.join(ROOT, "paper_2203_10000_amd", "csrc", "pairloop.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


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


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(labeling shards by points; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2203_10000_amd as sal
    import synth

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

    fp64 = None
    if args.fp64_steps > 0:
        lab64 = torch.empty_like(labels)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.fp64_steps):
            sal.label_points(ctx, ss, cen, precision="fp64", out=lab64)
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t1
        fp64 = {"value": pairs * args.fp64_steps / w64 / 1e9, "unit": "G pairs/s",
                "ms_per_step": 1e3 * w64 / args.fp64_steps, "steps": args.fp64_steps,
                "labels_equal_fp32_form": bool(torch.equal(lab64, labels))}

    achieved = FLOPS_PER_PAIR * pairs / (ms_pairloop * 1e-3) / 1e12
    traffic = hbm_traffic(pairs)
    roofline = {"bound": "alu", "kernel": "k_pairloop_f32<1>", "achieved": round(achieved, 2),
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
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
