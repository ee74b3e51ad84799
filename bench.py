#!/usr/bin/env python3
"""Benchmark of the LSG-CPD hot path on one MI355X.

One step = one full registration (lsgcpd_register) of the LiDAR-like pair
(100,000 target x 50,000 source points, the largest single-GPU workload):
target normals (20-NN PCA), target records, initial sigma^2, then 50 EM
iterations of E step + SE(3) M step.  Inputs are resident in HBM before the
timed region.

Prints one JSON line:
  value       = dense-equivalent E-step pair evaluations per second of the
                whole step: M * N * 50 / wall time of the step (normals and M
                steps included).  Every E step computes the posterior over all
                M N pairs; the pairs whose exponential is proven to be an exact
                float32 zero are counted but not evaluated.  The rate of pairs
                actually evaluated is `estep.evaluated_pair_evals_per_s`.
  roofline    = the E-step pair kernel, timed live with HIP events on its
                stream over a second run of the same K steps (the events
                are kept out of the steps that give `value`), credited with
                the method's 38 flops per (target, source) pair it evaluates
                (residual 3, squared norm 5, plane term 5, their sum 2, the
                exponent 2, the normaliser 1, the 10 weighted features 20;
                pairs proven to hold exact-zero exponentials are dropped and
                not credited), in FP64, against the 78.6 TFLOP/s FP64
                vector peak of MI355X; traffic = HBM bytes per launch from the
                committed rocprofv3 counter summary of the same kernel source
  cpu_baseline= the FP64 C oracle (one full E step of the same pair) on the
                host cores; the same oracle E step also gives `parity`, the
                largest error of the GPU's 86 statistics against it
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 38          # the method's flops per evaluated (m, n) pair
PEAK_FP64 = 78.6e12          # MI355X FP64 vector, FLOP/s
EM_ITERS = 50


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--backend", default="scalar", choices=["scalar", "dense", "lds", "mfma"],
                    help="pair-kernel back end (dense: scalar, every pair evaluated)")
    ap.add_argument("--workload", default="lidar_100000x50000",
                    choices=["rgbd_20000x20000", "lidar_100000x50000", "range_scanner_2000x2000",
                             "batch256", "batch256_small", "depth_cf_20000x20000",
                             "proposal1024"],
                    help="synthetic pair (the default is the benchmark's workload); batch256: "
                         "256 scene pairs of 1,000-30,000 points registered as one batch; "
                         "batch256_small: 256 pairs of 500-3,000 points; depth_cf: a depth-camera "
                         "pair registered with confidence filtering and truncation; "
                         "proposal1024: 1,024 scene pairs at rotations uniform on SO(3), "
                         "registered from the learned proposal (24-start fallback) against "
                         "plain single-pair registrations")
    ap.add_argument("--bf16", action="store_true",
                    help="single-pair workloads: LSGCPD_BF16_CROSS (matrix-core exponent in "
                         "the E steps whose error bound allows it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="batch workloads: skip the one-by-one registrations")
    ap.add_argument("--cpu-report", action="store_true",
                    help="only time the FP64 C oracle's E step on the three single-pair "
                         "workloads (all host cores and one) and a full 2,000-point "
                         "registration; no GPU")
    ap.add_argument("--traffic", type=str, default=None,
                    help="JSON file with measured HBM bytes per pair-kernel launch "
                         "(default: profiles/estep_pairs_<workload>_traffic.json)")
    ap.add_argument("--no-gpu-clock", action="store_true",
                    help="skip the rocm-smi clock query (under a profiler: rocm-smi starts a "
                         "second interpreter through its launcher)")
    ap.add_argument("--copy-kernel", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--traffic-record", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH",
                                                          "COPY_WRITE"),
                    help="only write profiles/estep_pairs_<workload>_traffic.json from four "
                         "rocprofv3 --pmc output folders: FETCH_SIZE and WRITE_SIZE of a bench "
                         "run of the workload, then of --copy-kernel 256")
    return ap.parse_args()


def measured_traffic(path):
    """HBM bytes per pair-kernel launch from the committed counter summary, or
    None when there is none or a source it depends on (the kernel, the host
    code that sizes its work items, and the point order that shapes its
    groups and tiles) changed since it was taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    srcs = rec.get("sources") or [{"path": rec.get("source", ""),
                                   "sha256": rec.get("source_sha256")}]
    for s in srcs:
        f = os.path.join(ROOT, s.get("path", ""))
        if not os.path.exists(f):
            return None
        if hashlib.sha256(open(f, "rb").read()).hexdigest() != s.get("sha256"):
            return None
    return rec.get("bytes_per_launch")


TRAFFIC_SOURCES = ["paper_2103_15039_amd/csrc/estep.hip", "paper_2103_15039_amd/csrc/api.hip",
                   "paper_2103_15039_amd/csrc/order.hip"]
PAIR_KERNEL = "estep_pairs_items"


def pmc_per_dispatch(folder, kernel_substring=None, largest=False):
    """Mean counter value per dispatch (KiB) from a rocprofv3 --pmc CSV
    folder: over the dispatches of kernels whose name contains
    kernel_substring, or of the kernel with the largest value (largest)."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(folder, "**", "*counter_collection*.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    if not rows:
        raise SystemExit(f"no counter_collection CSV under {folder}")
    per = {}
    for r in rows:
        name = r.get("Kernel_Name", "")
        if kernel_substring and kernel_substring not in name:
            continue
        key = (name, r.get("Dispatch_Id"))
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    if largest:
        top = max(per.items(), key=lambda kv: kv[1])[0][0]
        per = {k: v for k, v in per.items() if k[0] == top}
    vals = list(per.values())
    return sum(vals) / len(vals), len(vals)


def traffic_record(a):
    """HBM bytes per pair-kernel launch: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) of the pair kernel, each scaled by bytes / counter of a plain
    copy of 256 MiB; keyed on the SHA-256 of the kernel's and the plan's
    sources."""
    import hashlib
    fetch, nf = pmc_per_dispatch(a.traffic_record[0], PAIR_KERNEL)
    write, nw = pmc_per_dispatch(a.traffic_record[1], PAIR_KERNEL)
    cf, _ = pmc_per_dispatch(a.traffic_record[2], largest=True)
    cw, _ = pmc_per_dispatch(a.traffic_record[3], largest=True)
    copy_bytes = 256 * (1 << 20)
    fs, ws = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    rec = {"kernel": PAIR_KERNEL, "workload": a.workload,
           "bytes_per_launch": fetch * 1024.0 * fs + write * 1024.0 * ws,
           "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write,
           "dispatches": [nf, nw], "fetch_scale": fs, "write_scale": ws,
           "sources": [{"path": f, "sha256": hashlib.sha256(
               open(os.path.join(ROOT, f), "rb").read()).hexdigest()} for f in TRAFFIC_SOURCES]}
    out = os.path.join(ROOT, "profiles", f"estep_pairs_{a.workload}_traffic.json")
    json.dump(rec, open(out, "w"), indent=1)
    print(json.dumps(rec), flush=True)


def rot_err_deg(R, R_gt):
    """Angle of R_gt^T R in degrees, by atan2 of its sine and cosine (accurate
    near 0, where arccos of the trace is not)."""
    import numpy as np
    A = np.asarray(R_gt, dtype=np.float64).T @ np.asarray(R, dtype=np.float64)
    s = 0.5 * np.linalg.norm([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    c = 0.5 * (np.trace(A) - 1.0)
    return float(np.degrees(np.arctan2(s, c)))


def copy_kernel(mib):
    """A plain elementwise copy (read MIB MiB, write MIB MiB), three launches,
    for scaling the HBM byte counters of a profiler run."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_kernel_bytes_read": n * 4, "copy_kernel_bytes_written": n * 4,
                      "launches": 3}), flush=True)


def gpu_clock():
    """Shader and memory clocks as rocm-smi reports them (best effort; None if
    rocm-smi is unavailable)."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True,
                           text=True, timeout=30)
        j = json.loads(r.stdout)
        card = j[sorted(j)[0]]
        return {k: v for k, v in card.items() if "sclk" in k.lower() or "mclk" in k.lower()}
    except Exception:
        return None


def launch_stats(us, per_step):
    """Median, p10 and p90 of per-E-step times over EM iterations 2..50 of
    every timed registration (the first E step of each is left out)."""
    import numpy as np
    us = np.asarray(us)
    keep = us[np.arange(len(us)) % per_step != 0] if len(us) else us
    if len(keep) == 0:
        return None
    return {"median": float(np.median(keep)), "p10": float(np.percentile(keep, 10)),
            "p90": float(np.percentile(keep, 90)), "n": int(len(keep))}


# Pose offset and sigma^2 of the parity E step: a pose 0.01 deg / 1 mm off
# the ground truth and a sigma^2 of the order a registration of the workload
# ends on, where the exact culling drops most pairs (the late, culled regime).
PARITY_SIGMA2 = {"rgbd_20000x20000": 1.3e-3, "lidar_100000x50000": 7.5e-3,
                 "range_scanner_2000x2000": 2.0e-5}


def parity_inputs(p, workload):
    """Seeded E-step inputs shared by the GPU and the oracle: unit normals and
    penalties drawn at random (an E step's cost and its error do not depend on
    where they come from), a pose near the ground truth, a late sigma^2."""
    import numpy as np
    import datagen
    M = len(p.Y)
    rng = np.random.default_rng([210315039, 99])
    nrm = rng.normal(size=(M, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    al = rng.uniform(0.0, 30.0, size=M)
    R = datagen.random_rotation(rng, np.radians(0.01)) @ p.R_gt
    t = p.t_gt + rng.uniform(-1e-3, 1e-3, size=3)
    return (nrm.astype(np.float32), al.astype(np.float32), R, t,
            PARITY_SIGMA2.get(workload, 1e-3))


def cpu_baseline(p, nrm, alpha, R, t, s2, gpu):
    """The oracle's C E step (FP64, OpenMP over sources): one full E step of
    the same pair, timed; its 86 statistics against the GPU's at the same
    inputs give the parity record (error per statistic relative to the sum of
    the magnitudes of its terms, and the NLL's relative error)."""
    import numpy as np
    from oracle import c_oracle as CO
    from oracle import lsgcpd_oracle as O
    if not os.path.exists(CO.LIB):
        CO.build()
    V = O.working_volume(p.Y)
    t0 = time.perf_counter()
    cols, ks = CO.estep_columns(p.X, p.Y, nrm, alpha, R, t, s2, w0=0.1, V=V)
    dt = time.perf_counter() - t0
    N = len(p.X)
    pairs = N * len(p.Y)
    gamma = (2 * np.pi * s2) ** 1.5 / V
    terms = [float(np.sum(np.log(ks + gamma))), float(np.sum(gamma / (ks + gamma))),
             N * float(np.log(0.1))]
    ref = O.lifted_stats(cols, p.X, terms)
    W = cols.A - cols.p[:, None, None] * np.eye(3)[None]
    ab = O.Columns(p=np.abs(cols.p), A=np.abs(W) + np.abs(cols.p)[:, None, None] * np.eye(3)[None],
                   B=np.abs(cols.B), C=np.abs(cols.C), b=None, c=None)
    scale = O.lifted_stats(ab, np.abs(p.X.astype(np.float64)))
    scale[83:] = np.abs(ref[83:]) + N
    rel = np.abs(np.asarray(gpu.stats) - ref) / np.maximum(scale, 1e-300)
    nll = -(ref[85] + ref[83] - 1.5 * N * np.log(2 * np.pi * s2))
    base = {"value": pairs / dt, "unit": "pair-evals/s", "cores": CO.threads(),
            "kind": "oracle",
            "sample": f"one full FP64 E step ({len(p.Y)} x {N} pairs, posterior and "
                      f"per-source sums) of the benchmark pair near its ground-truth pose at "
                      f"sigma^2 = {s2:g}, {dt:.2f} s"}
    parity = {"what": "86 E-step statistics of lsgcpd_estep vs the FP64 C oracle, same inputs "
                      f"(pose 0.01 deg / 1 mm off the truth, sigma^2 = {s2:g}, seeded normals)",
              "max_err_rel_to_sum_abs_terms": float(rel.max()),
              "worst_stat": int(np.argmax(rel)),
              "nll_rel_err": abs(gpu.nll - nll) / abs(nll),
              "sumP_rel_err": abs(gpu.sumP - ref[9]) / max(abs(ref[9]), 1e-300),
              "bar": 2e-6}
    return base, parity


def batch_main(a, nmin=1000, nmax=30000):
    """256 pairs of box/sphere/plane scenes, M and N log-uniform in
    [nmin, nmax], rotations up to 60 deg: pairs registered per second by
    lsgcpd_register_batch (the timed steps) next to the same pairs registered
    one by one with lsgcpd_register (one untimed-for-value pass), and the
    success rate (rotation error < 1 deg) of both."""
    import numpy as np
    import torch
    import datagen
    import paper_2103_15039_amd as L

    pairs = datagen.batch_pairs(256, trial=0, nmin=nmin, nmax=nmax)
    args = [(torch.from_numpy(p.X).cuda(), torch.from_numpy(p.Y).cuda()) for p in pairs]
    kw = dict(k=10, alpha_max=30.0, lam=0.2, w0=0.1, max_iter=EM_ITERS)
    torch.cuda.synchronize()
    for _ in range(a.warmup):
        L.register_batch(args, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        res = L.register_batch(args, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L.profile_enable(True)          # kernel timing: the same steps again
    L.profile_read(reset=True)
    for _ in range(a.steps):
        L.register_batch(args, **kw)
    torch.cuda.synchronize()
    prof = L.profile_read(reset=True)
    L.profile_enable(False)
    single, dt_single = None, None
    if not a.no_plain:
        t1 = time.perf_counter()
        single = [L.register(X, Y, **kw) for X, Y in args]
        torch.cuda.synchronize()
        dt_single = time.perf_counter() - t1

    def ok(rs):
        return float(np.mean([rot_err_deg(r.R, p.R_gt) < 1.0 for r, p in zip(rs, pairs)]))
    k_ms = prof["pair_kernel_ms"] / max(prof["launches"], 1)
    evaluated = prof["evaluated_pairs"] / max(prof["launches"], 1)
    achieved = FLOPS_PER_PAIR * evaluated / (k_ms * 1e-3)
    value = len(pairs) * a.steps / dt
    mn = sum(len(p.X) * len(p.Y) for p in pairs)
    out = {
        "metric": "pairs registered/s",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "pairs": len(pairs),
                   "points": f"{nmin}-{nmax} log-uniform",
                   "em_iters": EM_ITERS, "knn": 10, "sum_MN": mn},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None},
        "plain": None if single is None else {
            "pairs_per_s": len(pairs) / dt_single, "ms": dt_single * 1e3,
            "success_rate": ok(single),
            "successful_pairs_per_s": ok(single) * len(pairs) / dt_single},
        "batched": {"success_rate": ok(res),
                    "successful_pairs_per_s": ok(res) * value,
                    "speedup_vs_plain": None if single is None else value * dt_single / len(pairs),
                    "estep_pair_evals_per_s": mn * EM_ITERS * a.steps / dt,
                    "pair_kernel_ms": k_ms, "evaluated_frac": evaluated / mn},
    }
    print(json.dumps(out), flush=True)


def cf_main(a):
    """Confidence filtering (Sec. 3.3) on a depth-camera pair (20,000 x 20,000
    points, depth noise growing with the square of the depth): registrations
    per second and rotation error against the ground truth of the plain
    method (w0 = 0.1), of w0 from the outlier ratio (eta = 0.02), of confidence
    filtering without truncation (w0 = 0.1, and w0 from eta), and with
    truncation at several confidence
    thresholds.  The timed steps (value) are confidence filtering with
    truncation at the middle threshold; every variant is timed the same way."""
    import numpy as np
    import torch
    import datagen
    import paper_2103_15039_amd as L

    trials = [datagen.depth_pair(trial=t) for t in range(3)]
    dev = [(torch.from_numpy(p.X).cuda(), torch.from_numpy(p.Y).cuda()) for p in trials]
    conf = [(L.depth_confidence(X, datagen.DEPTH_ERROR, datagen.DEPTH_ERROR_MIN),
             L.depth_confidence(Y, datagen.DEPTH_ERROR, datagen.DEPTH_ERROR_MIN)) for X, Y in dev]
    kw = dict(k=20, alpha_max=30.0, lam=0.2, max_iter=EM_ITERS)
    variants = [("plain", dict(w0=0.1), None), ("eta", dict(eta=0.02), None),
                ("cf_w0", dict(w0=0.1), 0.0), ("cf", dict(eta=0.02), 0.0)] + \
               [(f"cf_trunc_{t}", dict(eta=0.02), t) for t in (0.03, 0.05, 0.08)]

    def run(i, extra, thr):
        X, Y = dev[i]
        if thr is None:
            return L.register(X, Y, **kw, **extra)
        return L.register_cf(X, Y, conf[i][0], conf[i][1], threshold=thr, **kw, **extra)

    out_var = {}
    for name, extra, thr in variants:
        for _ in range(a.warmup):
            run(0, extra, thr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            for i in range(len(dev)):
                r = run(i, extra, thr)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / (a.steps * len(dev))
        errs = [rot_err_deg(run(i, extra, thr).R, p.R_gt) for i, p in enumerate(trials)]
        last = run(0, extra, thr)
        out_var[name] = {"ms": dt * 1e3, "registrations_per_s": 1.0 / dt,
                         "rot_err_deg": errs, "rot_err_mean": float(np.mean(errs)),
                         "points_kept": [int(last.n_used), int(last.m_used)], "w0": last.w0}
        print(f"# {name}: {dt * 1e3:.2f} ms, rot err {np.mean(errs):.3f} deg", file=sys.stderr,
              flush=True)
    main_v = out_var["cf_trunc_0.05"]
    out = {
        "metric": "registrations/s",
        "value": main_v["registrations_per_s"],
        "unit": "registrations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": main_v["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "M": 20000, "N": 20000, "em_iters": EM_ITERS,
                   "knn": 20, "eta": 0.02, "threshold": 0.05, "depth_error": datagen.DEPTH_ERROR,
                   "trials": len(trials)},
        "variants": out_var,
    }
    print(json.dumps(out), flush=True)


def cpu_report():
    """The oracle on the host: one full FP64 E step of each single-pair
    workload with all cores (the LiDAR pair: 3 E steps), the RGB-D E step on
    one core (a 2,000-source slice, scaled), and the full 2,000 x 2,000
    registration (50 iterations, C E step)."""
    import platform
    import numpy as np
    import datagen
    from oracle import c_oracle as CO
    from oracle import lsgcpd_oracle as O
    CO.build()
    model = platform.processor()
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo")
                 if l.startswith("model name")][0]
    except Exception:
        pass
    allc = CO.threads()
    out = {"cpu_model": model, "threads": allc, "nproc": os.cpu_count(), "estep": {}}
    rng = np.random.default_rng(0)
    for name in ("range_scanner_2000x2000", "rgbd_20000x20000", "lidar_100000x50000"):
        p = datagen.WORKLOADS[name](trial=0)
        M, N = len(p.Y), len(p.X)
        nrm = rng.normal(size=(M, 3))
        nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
        al = rng.uniform(0.0, 30.0, size=M).astype(np.float32)
        R, t = np.eye(3), np.zeros(3)
        s2 = CO.sigma2_init(p.X, p.Y, R, t)
        V = O.working_volume(p.Y)
        reps = 3 if name.startswith("lidar") else 1
        CO.set_threads(allc)
        t0 = time.perf_counter()
        for _ in range(reps):
            CO.estep_columns(p.X, p.Y, nrm, al, R, t, s2, w0=0.1, V=V)
        dt = (time.perf_counter() - t0) / reps
        rec = {"pairs": M * N, "seconds": dt, "pair_evals_per_s_all_cores": M * N / dt}
        if name.startswith("rgbd"):
            CO.set_threads(1)
            Xs = p.X[:2000]
            t0 = time.perf_counter()
            CO.estep_columns(Xs, p.Y, nrm, al, R, t, s2, w0=0.1, V=V)
            d1 = time.perf_counter() - t0
            rec["pair_evals_per_s_one_core"] = M * len(Xs) / d1
            CO.set_threads(allc)
        out["estep"][name] = rec
        print(f"# {name}: {rec}", file=sys.stderr, flush=True)
    p = datagen.range_scanner_pair(trial=0)
    t0 = time.perf_counter()
    nrm, _, al = O.normals(p.Y, 10, 30.0, 0.2)
    fn = CO.register_columns_fn(p.X, p.Y, nrm.astype(np.float32), al.astype(np.float32), 0.1,
                                O.working_volume(p.Y))
    r = O.register(p.X, p.Y, k=10, max_iter=EM_ITERS, target_normals=nrm, target_alpha=al,
                   estep_columns=fn)
    out["register_range_scanner_2000x2000_s"] = time.perf_counter() - t0
    out["register_rot_err_deg"] = float(O.rotation_error_deg(r.R, p.R_gt))
    print(json.dumps(out), flush=True)


PROPOSAL_THETA = os.path.join(ROOT, "paper_2103_15039_amd", "proposal_theta.npy")


def proposal_main(a, npairs=1024, nsub=64, P=512, accepts=(0.1, 0.05)):
    """The learned initial pose (the benchmark spec's M2): 1,024 held-out scene pairs
    (2-3 primitives, M and N log-uniform in [1,000, 30,000], source rotation
    uniform on SO(3)).  Timed, in registrations per second and with the
    success rate (rotation error < 1 deg against the truth):
      * proposed: lsgcpd_register_proposed -- the encoder's poses for all
        pairs, EM from each in one batch, and for the pairs whose final sigma
        exceeds `accept` times the target's RMS radius, EM from the 4 sign
        changes of the principal axes, then the other 20 cube rotations
        (lowest NLL wins); at accept = 0.1 (value: on held-out pairs 0.5 % of
        the correct registrations end above it) and at 0.05 (nearly every
        pair takes the fallback: the most thorough setting);
      * plain: lsgcpd_register one pair at a time from the identity (all
        pairs);
      * plain, 24 starts: lsgcpd_register one pair at a time from each of the
        24 cube rotations (centroids aligned), lowest NLL kept -- the
        the benchmark spec's multi-start judge; timed on the first `nsub` pairs (its
        rate per pair is what is reported).
    EM: k = 10, 50 iterations at most, stopping when the relative NLL change
    falls below 1e-6, for every path."""
    import numpy as np
    import torch
    import datagen
    import paper_2103_15039_amd as L

    theta = torch.from_numpy(np.load(PROPOSAL_THETA).astype(np.float32)).cuda()
    pairs = datagen.proposal_pairs(npairs, split="eval", trial=0)
    dev = [(torch.from_numpy(p.X).cuda(), torch.from_numpy(p.Y).cuda()) for p in pairs]
    kw = dict(k=10, alpha_max=30.0, lam=0.2, w0=0.1, max_iter=EM_ITERS, tol=1e-6)

    def ok(rs, ps):
        return np.array([rot_err_deg(r.R, p.R_gt) < 1.0 for r, p in zip(rs, ps)])
    torch.cuda.synchronize()
    L.register_proposed(dev[:8], theta, P=P, accept=accepts[0], **kw)   # warm-up
    runs = {}
    for acc in accepts:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, fb = L.register_proposed(dev, theta, P=P, accept=acc, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        succ = ok(res, pairs)
        runs[acc] = {"pairs_per_s": npairs / dt, "s": dt, "success_rate": float(succ.mean()),
                     "successful_pairs_per_s": float(succ.mean()) * npairs / dt,
                     "fallback_rate": float(np.mean(fb)),
                     "success_on_the_24_start_subset": float(succ[:nsub].mean())}
    # the encoder alone: its poses and their error
    Xn, Yn, nm = L.proposal_inputs(dev, P)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pose = L.proposal_forward(theta, Xn, Yn, nm)
    torch.cuda.synchronize()
    dt_fwd = time.perf_counter() - t1
    pose = pose.cpu().numpy()
    prop_err = np.array([rot_err_deg(pose[i, :9].reshape(3, 3), p.R_gt)
                         for i, p in enumerate(pairs)])
    t2 = time.perf_counter()
    plain = [L.register(X, Y, **kw) for X, Y in dev]
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t2
    succ_plain = ok(plain, pairs)
    G = cube_rotations()
    t3 = time.perf_counter()
    best = []
    for X, Y in dev[:nsub]:
        mx = X.double().mean(0).cpu().numpy()
        my = Y.double().mean(0).cpu().numpy()
        rs = [L.register(X, Y, R0=g, t0=my - g @ mx, **kw) for g in G]
        best.append(min(rs, key=lambda r: r.nll[-1]))
    torch.cuda.synchronize()
    dt_multi = time.perf_counter() - t3
    succ_multi = ok(best, pairs[:nsub])
    rate_multi = nsub / dt_multi
    main_run = runs[accepts[0]]
    out = {
        "metric": "pairs registered/s at rotation error < 1 deg",
        "value": main_run["successful_pairs_per_s"],
        "unit": "successful pairs/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": main_run["s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "proposal1024", "pairs": npairs,
                   "points": "1000-30000 log-uniform", "rotation": "uniform on SO(3)",
                   "encoder_points": P, "accept_sigma_over_radius": accepts[0],
                   "em_max_iters": EM_ITERS, "em_tol": 1e-6, "knn": 10},
        "proposed": {f"accept_{acc}": r for acc, r in runs.items()},
        "encoder": {"ms_all_pairs": dt_fwd * 1e3,
                    "rot_err_deg_median": float(np.median(prop_err)),
                    "within_30deg": float(np.mean(prop_err < 30)),
                    "within_60deg": float(np.mean(prop_err < 60))},
        "plain_identity": {"pairs_per_s": npairs / dt_plain,
                           "success_rate": float(succ_plain.mean()),
                           "successful_pairs_per_s": float(succ_plain.mean()) * npairs / dt_plain},
        "plain_24_starts": {"pairs_per_s": rate_multi, "success_rate": float(succ_multi.mean()),
                            "pairs_timed": nsub,
                            "successful_pairs_per_s": float(succ_multi.mean()) * rate_multi},
        "proposed_over_plain_24_starts": {
            f"accept_{acc}": {"pairs_per_s": r["pairs_per_s"] / rate_multi,
                              "successful_pairs_per_s":
                                  r["successful_pairs_per_s"] / max(succ_multi.mean() * rate_multi,
                                                                    1e-30)}
            for acc, r in runs.items()},
    }
    print(json.dumps(out), flush=True)


def cube_rotations():
    """The 24 rotations of the cube (signed permutation matrices, det +1)."""
    import itertools
    import numpy as np
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1.0, -1.0), repeat=3):
            R = np.zeros((3, 3))
            for r in range(3):
                R[r, perm[r]] = signs[r]
            if np.linalg.det(R) > 0:
                out.append(R)
    return out


def main():
    a = parse()
    if a.cpu_report:
        cpu_report()
        return
    if a.copy_kernel:
        copy_kernel(a.copy_kernel)
        return
    if a.traffic_record:
        traffic_record(a)
        return
    if a.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {a.gpus}); "
              "sharding across GPUs is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)
    if a.workload == "batch256":
        batch_main(a)
        return
    if a.workload == "batch256_small":
        batch_main(a, 500, 3000)
        return
    if a.workload.startswith("depth_cf"):
        cf_main(a)
        return
    if a.workload == "proposal1024":
        proposal_main(a)
        return
    import numpy as np
    import torch
    import datagen
    import paper_2103_15039_amd as L

    p = datagen.WORKLOADS[a.workload](trial=0)
    M, N = len(p.Y), len(p.X)
    knn = 10 if a.workload.startswith("range") else 20
    X = torch.from_numpy(p.X).cuda()
    Y = torch.from_numpy(p.Y).cuda()
    kw = dict(k=knn, alpha_max=30.0, lam=0.2, w0=0.1, max_iter=EM_ITERS, backend=a.backend,
              bf16=a.bf16)
    torch.cuda.synchronize()
    for _ in range(a.warmup):
        L.register(X, Y, **kw)
    torch.cuda.synchronize()
    # value: K steps as a user runs them; then the same K steps again with
    # HIP events around every pair kernel and E step (the events themselves
    # cost about 3 us each on the stream, so they stay out of the first loop)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        r = L.register(X, Y, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L.profile_enable(True)
    L.profile_read(reset=True)
    t1 = time.perf_counter()
    for _ in range(a.steps):
        L.register(X, Y, **kw)
    torch.cuda.synchronize()
    dt_prof = time.perf_counter() - t1
    pair_us, estep_us = L.profile_launches()
    prof = L.profile_read(reset=True)
    L.profile_enable(False)
    est = launch_stats(estep_us, EM_ITERS)
    pst = launch_stats(pair_us, EM_ITERS)

    pairs_per_step = M * N * EM_ITERS
    value = pairs_per_step * a.steps / dt
    k_ms = prof["pair_kernel_ms"] / max(prof["launches"], 1)
    e_ms = prof["estep_ms"] / max(prof["launches"], 1)
    evaluated = prof["evaluated_pairs"] / max(prof["launches"], 1)
    achieved = FLOPS_PER_PAIR * evaluated / (k_ms * 1e-3)
    traffic = measured_traffic(a.traffic or os.path.join(
        ROOT, "profiles", f"estep_pairs_{a.workload}_traffic.json"))
    rot_err = rot_err_deg(r.R, p.R_gt)
    out = {
        "metric": "E-step pair-evals/s",
        "value": value,
        "unit": "pair-evals/s (dense-equivalent: M*N per E step)",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "M": M, "N": N, "em_iters": EM_ITERS,
                   "knn": knn, "alpha_max": 30.0, "lambda": 0.2, "w0": 0.1,
                   "pair_kernel": a.backend, "bf16_cross": a.bf16},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": traffic},
        "estep": {"pair_kernel_ms": k_ms, "estep_ms": e_ms,
                  "ms_per_step_with_events": dt_prof / a.steps * 1e3,
                  "estep_us_iters_2_50": est, "pair_kernel_us_iters_2_50": pst,
                  "dense_equiv_pair_evals_per_s_median_estep":
                      M * N / (est["median"] * 1e-6) if est else None,
                  "gpu_clock": None if a.no_gpu_clock else gpu_clock(),
                  "evaluated_frac": evaluated / (M * N),
                  "evaluated_pair_evals_per_s": evaluated * EM_ITERS * a.steps / dt,
                  "evaluated_pair_evals_per_s_pair_kernel": evaluated / (k_ms * 1e-3),
                  "dense_equiv_pair_evals_per_s_pair_kernel": M * N / (k_ms * 1e-3),
                  "dense_equiv_pair_evals_per_s_estep": M * N / (e_ms * 1e-3),
                  "launches_timed": prof["launches"]},
        "result": {"rot_err_deg_vs_truth": rot_err, "iters": r.iters, "sigma2": r.sigma2,
                   "bf16_estep_count": r.bf16_steps},
    }
    if not a.no_cpu_baseline:
        nrm, al, Rp, tp, s2p = parity_inputs(p, a.workload)
        g = L.estep(X, Y, torch.from_numpy(nrm).cuda(), torch.from_numpy(al).cuda(), Rp, tp,
                    s2p, w0=0.1)
        torch.cuda.synchronize()
        out["cpu_baseline"], out["parity"] = cpu_baseline(p, nrm, al, Rp, tp, s2p, g)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
