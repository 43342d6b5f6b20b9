#!/usr/bin/env python3
"""Throughput of the Vecchia hot path on one MI355X.

One step = factor (Eq. (2) for every point + dense block) + forward
(Alg. 1, batch by batch) + logdet, on the workload's point cloud resident in
HBM.  The host graph build runs once before timing (it depends only on the
points) and is reported separately.  Prints ONE JSON line on stdout; progress
goes to stderr.

Default workload: 2^26 points, 90% uniform in [0,1]^3 + 10% Gaussian clumps
of width 1e-3, k = 32, squared-exponential kernel ell = 0.02, nugget 1e-6,
FP32 storage with FP64 pivots and logdet.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
VALU_PEAK_TFLOPS = 78.6        # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz: FP32 unpacked = FP64 FMA rate
VALU_PEAK_TLANEOPS = 39.32     # 256 CU x 64 lanes x 2.4 GHz: one VALU lane-operation (an FMA counts one)
METRIC = "points/sec Vecchia factor+forward+logdet (k=16,32); p50/p99 req latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def eval_flops(kind):
    # flops of one kernel evaluation from three coordinate differences:
    # r^2 (3 sub, 3 mul, 2 add) + scaling and amplitude; exp and sqrt count 1 each
    return {0: 12, 1: 14, 2: 11}[kind]


def factor_flops_per_point(k, kind, refine):
    """Algorithmic flops of Eq. (2) for one point with k neighbours."""
    evals = k * (k + 1) // 2 + k                    # lower K_cc + k_ci
    chol = k ** 3 / 3.0 + k * k / 2.0               # right-looking Cholesky
    solves = 2.0 * k * k + 2 * k                    # L y = k_ci, L^T b = y, sigma^2
    total = evals * eval_flops(kind) + chol + solves
    if refine:
        total += (k * (k + 1) // 2) * eval_flops(kind) + 2.0 * k * k   # residual k - K b
        total += 2.0 * k * k + 2 * k                                   # correction solves, k.b
    return total


def factor_laneops_per_point(k, kind, refine):
    """Algorithmic VALU lane-operations of Eq. (2) for one point with k
    neighbours, one FMA or one transcendental counting one: k(k+1)/2 kernel
    evaluations of K_cc (about 11 operations for the squared exponential, 16
    for Matern-3/2, 12 for the exponential), the Cholesky (k^3/6 FMA plus
    k^2/2 + 8k for scaling, pivots and reciprocals), the two triangular solves
    and sigma^2 (k^2 + k).  The refinement step of the float pass adds the
    residual's kernel evaluations and about 2.5 k^2 more."""
    per_eval = {0: 12, 1: 16, 2: 11}[kind]
    total = k * (k + 1) // 2 * per_eval + k ** 3 / 6.0 + k * k / 2.0 + 8 * k + k * k + k
    if refine:
        total += k * (k + 1) // 2 * per_eval + 2.5 * k * k
    return total


def factor_bytes_per_point(k, esz):
    # neighbour indices, gathered neighbour coordinates, own coordinates, b and sigma out
    return 4 * k + 3 * esz * k + 3 * esz + esz * k + esz


def precision_note(precision, n_redo, ns):
    if precision != 1:
        return "fp64 throughout"
    head = "fp32 storage of b, sigma, v; forward in fp32; logdet in fp64 (compensated); "
    if n_redo == ns:
        return head + ("factor arithmetic in fp64 for every point: the sampled policy found that float kernel "
                       "values cannot resolve these conditional variances")
    return head + ("factor in fp32 with fp64 pivots and one refinement step; %d of %d points recomputed in fp64"
                   % (n_redo, ns))


def apply_bytes_per_point(k, esz):
    # neighbour index + coefficient + gathered v per neighbour, sigma, xi/v in, v/xi out
    return 4 * k + esz * k + esz * k + 3 * esz


def kernel_sources(precision_name, kp):
    """Source files that define the factor kernel of this precision and width,
    and the graph builder that lays out its neighbour rows (their order sets
    the kernel's gather pattern, hence its traffic)."""
    csrc = os.path.join(ROOT, "paper_2606_11402_amd", "csrc")
    return [os.path.join(csrc, f) for f in
            ("common.h", "lanes.h", "factor_kernel.h", "factor_%s_k%d.hip" % (precision_name, kp), "graph.cpp")]


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel, workload, digest):
    """HBM bytes per launch of `kernel` on `workload` from a committed counter
    summary (profiles/traffic_*.txt, lines "key: value"), or None when there is
    none or it was taken on other kernel sources than the current ones."""
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.txt"))):
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith((" ", "#")):
                    a, b = line.split(":", 1)
                    kv[a.strip()] = b.strip()
        if kv.get("kernel") != kernel or kv.get("workload") != workload:
            continue
        if kv.get("source_digest") != digest:
            log("traffic summary %s was taken on other kernel sources; traffic = null" % os.path.basename(path))
            return None
        try:
            return {"fetch_bytes": float(kv["fetch_bytes_per_launch"]),
                    "write_bytes": float(kv["write_bytes_per_launch"]),
                    "copy_scale_fetch": float(kv["copy_scale_fetch"]),
                    "copy_scale_write": float(kv["copy_scale_write"]),
                    "summary": "profiles/" + os.path.basename(path)}
        except (KeyError, ValueError):
            return None
    return None


def calibrate_copy():
    """One plain 1 GiB device-to-device copy (three times), for scaling the
    FETCH_SIZE / WRITE_SIZE counters: the copy reads and writes 2^30 bytes."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="override N (default: the workload's)")
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--threads", type=int, default=0, help="host threads for the graph build")
    ap.add_argument("--host-knn", action="store_true",
                    help="run the graph's neighbour search on the host instead of the device")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled oracle check")
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--cpu-passes", type=int, default=24)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparisons (FP64 path on the same workload, k=16 radial in both precisions)")
    ap.add_argument("--serve-requests", type=int, default=128,
                    help="requests of the serving measurement (0 skips it)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the gradient configuration (2^22 radial, k = 16) and print its record")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures the Vecchia hot path on one GPU only; runs on several GPUs are not "
              "part of this build (see DESIGN.md for how the path would shard).", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.adjoint_only:
        import torch
        print(json.dumps({"adjoint_radial_2e22": adjoint_step(args.steps, torch.device("cuda:0"))}), flush=True)
        return

    import workloads
    w = workloads.WORKLOADS[args.workload]
    n = args.n or w.n
    k = args.k or w.k
    n0 = w.n0
    # the CPU baseline runs first, before anything initialises the GPU, so
    # that its forked worker processes inherit no device state
    cpu = None if args.no_cpu_baseline else cpu_baseline(w, k, n0, args.cpu_sample, args.cpu_passes)

    import numpy as np
    import torch

    from paper_2606_11402_amd import FP32, FP64, Factor, Graph, KernelParams
    from paper_2606_11402_amd import vecchia as vmod

    precision = FP32 if "fp32" in w.precisions else FP64
    esz = 4 if precision == FP32 else 8
    dev = torch.device("cuda:0")
    kern = KernelParams(w.kind, w.sigma, w.ell, w.nugget)

    log("workload %s: N=%d k=%d n0=%d, generating points" % (w.name, n, k, n0))
    t = time.time()
    x = w.points(n)
    xi_in = w.xi(n)
    log("points ready in %.1fs; building graph on the host" % (time.time() - t))
    t = time.time()
    g = Graph(x, k, n0, n_threads=args.threads, knn_device=None if args.host_knn else "cuda:0")
    graph_s = time.time() - t
    graph_phases = {a: round(b, 2) for a, b in g.build_times().items()}
    if g.knn_seconds is not None:
        graph_phases["neighbours"] = round(g.knn_seconds, 2)      # device search incl. transfers
        graph_phases["split"] = {a: round(b, 2) for a, b in g.split_seconds.items()}
    log("graph: %.1fs %s, %d levels (neighbour search on the %s)" % (graph_s, graph_phases, g.n_levels,
                                                                      "host" if args.host_knn else "device"))
    t = time.time()
    dg = g.to_device(precision, dev)
    dt = dg.dtype
    xi = torch.from_numpy(g.to_storage(xi_in)).to(dt).to(dev)
    del x
    v = torch.empty(n, dtype=dt, device=dev)
    ld = torch.empty(1, dtype=torch.float64, device=dev)
    fac = Factor(dg, kern)
    fac.status()
    n_bad, n_redo = fac.counts()
    upload_s = time.time() - t
    log("uploaded and factored once in %.1fs" % upload_s)

    def step():
        fac.refactor()
        fac.forward(xi, out=v)
        fac.logdet(out=ld)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fac.status()

    # ---- timed region: K whole steps, no per-kernel instrumentation
    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step / 1e3)
    log("%.3f ms/step, %.3e points/s" % (ms_per_step, value))

    # ---- same steps with HIP events around every launch (per-kernel times)
    vmod.profile_reset()
    vmod.profile_enable(True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    inv_out = torch.empty_like(v)
    for _ in range(args.steps):
        fac.inverse(v, out=inv_out)
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    prof = vmod.profile_read()
    vmod.profile_enable(False)
    log("per-kernel totals:", {a: (round(b[0], 3), b[1]) for a, b in prof.items()})

    # ---- forward + logdet alone without per-launch events: two events on the
    # stream the library launches on (torch's current stream) around K passes
    fac.forward(xi, out=v)
    fac.logdet(out=ld)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        fac.forward(xi, out=v)
        fac.logdet(out=ld)
    ev1.record()
    torch.cuda.synchronize()
    fl_wall_ms = ev0.elapsed_time(ev1) / args.steps

    # ---- the fused on-the-fly forward (Alg. 1 as written, nothing stored per
    # point) with its logdet, on the same points, graph and white noise
    fused = fused_forward_run(dg, kern, xi, v, ld, args.steps, n)

    ns = n - n0
    steps = args.steps
    avg = lambda name: prof[name][0] / prof[name][1] if name in prof else 0.0
    sparse_ms, redo_ms, probe_ms = avg("factor_sparse"), avg("factor_redo"), avg("factor_probe")
    n_bad, n_redo = fac.counts()
    # the dominant factor kernel: the float pass (every point, with refinement)
    # or the double pass (the recomputed points, no refinement)
    if redo_ms > sparse_ms:
        dom, f_ms, units = "factor_redo", redo_ms, n_redo
        fpp = factor_flops_per_point(k, w.kind, False)
        lpp = factor_laneops_per_point(k, w.kind, False)
        dom_desc = "factor_redo (Eq. 2 in FP64 for the points float cannot resolve: gather, K_cc, Cholesky, solves)"
    else:
        dom, f_ms, units = "factor_sparse", sparse_ms, ns
        fpp = factor_flops_per_point(k, w.kind, precision == FP32)
        lpp = factor_laneops_per_point(k, w.kind, precision == FP32)
        dom_desc = "factor_sparse (Eq. 2 per point: gather, K_cc, Cholesky, solves, refinement)"
    flops = fpp * units
    f_tflops = flops / (f_ms * 1e-3) / 1e12 if f_ms > 0 else 0.0
    f_tlops = lpp * units / (f_ms * 1e-3) / 1e12 if f_ms > 0 else 0.0
    fwd_ms = sum(t for name, (t, _) in prof.items() if name.startswith("forward_")) / steps
    ld_ms = prof["logdet"][0] / prof["logdet"][1]
    inv_ms = (prof["inverse_sparse"][0] + prof.get("inverse_dense", (0.0, 0))[0]) / steps
    inv_sparse_ms = prof["inverse_sparse"][0] / prof["inverse_sparse"][1]
    bpp = apply_bytes_per_point(k, esz)
    fwd_gbs = bpp * ns / (fwd_ms * 1e-3) / 1e9
    ldbytes = 8 * ((ns + 63) // 64)
    fl_gbs = (bpp * ns + ldbytes) / (fl_wall_ms * 1e-3) / 1e9
    inv_gbs = bpp * ns / (inv_sparse_ms * 1e-3) / 1e9
    levels_ms = sum(t for name, (t, _) in prof.items()
                    if name.startswith("forward_") and name != "forward_dense") / steps
    kp = 8 if k <= 8 else (16 if k <= 16 else (32 if k <= 32 else 64))
    digest = source_digest(kernel_sources("f32" if precision == FP32 else "f64", kp))
    tr = read_traffic(dom, w.name if args.n is None and args.k is None else None, digest)
    traffic, traffic_detail = None, None
    if tr is not None:
        traffic = tr["fetch_bytes"] + tr["write_bytes"]
        traffic_detail = {"fetch_bytes": tr["fetch_bytes"], "write_bytes": tr["write_bytes"],
                          "copy_scale_fetch": tr["copy_scale_fetch"], "copy_scale_write": tr["copy_scale_write"],
                          "algorithmic_bytes": factor_bytes_per_point(k, esz) * units, "summary": tr["summary"]}

    roofline = {
        "kernel": dom_desc,
        "bound": "alu", "achieved": round(f_tlops, 3), "peak": VALU_PEAK_TLANEOPS, "unit": "Tlane-op/s",
        "frac": round(f_tlops / VALU_PEAK_TLANEOPS, 4), "traffic": traffic,
        "laneops_per_point": lpp, "points_per_launch": units,
        "avg_launch_ms": round(f_ms, 4), "source_digest": digest, "traffic_detail": traffic_detail,
        "flop_count": {"flops_per_point": fpp, "achieved_tflops": round(f_tflops, 3),
                       "peak_tflops": VALU_PEAK_TFLOPS, "frac": round(f_tflops / VALU_PEAK_TFLOPS, 4),
                       "note": "second count: FMA = 2 flops, each exp/sqrt = its evaluation cost"},
    }
    others = {
        "forward": {"bound": "hbm", "achieved": round(fwd_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(fwd_gbs / HBM_PEAK_GBS, 4), "bytes_per_point": bpp,
                    "ms_per_forward": round(fwd_ms, 4), "launches_per_forward": sum(c for name, (_, c) in prof.items()
                                                                if name.startswith("forward_")) // steps},
        "forward+logdet": {"bound": "hbm", "achieved": round(fl_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(fl_gbs / HBM_PEAK_GBS, 4), "ms": round(fl_wall_ms, 4),
                           "ms_with_per_launch_events": round(fwd_ms + ld_ms, 4),
                           "small_batch_runs_ms": round(prof.get("forward_run", (0.0, 0))[0] / steps, 4),
                           "per_batch_launches_ms": round(prof.get("forward_level", (0.0, 0))[0] / steps, 4)},
        "inverse_sparse": {"bound": "hbm", "achieved": round(inv_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(inv_gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(inv_sparse_ms, 4)},
    }

    out = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": ("f32+f64" if n_redo > 0 else "f32") if precision == FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "k": k, "n0": n0, "kernel": ["EXP", "M32", "SE"][w.kind],
                   "ell": w.ell, "sigma": w.sigma, "nugget": w.nugget,
                   "precision": precision_note(precision, n_redo, ns), "levels": g.n_levels,
                   "points_recomputed_fp64": n_redo},
        "roofline": roofline,
        "rooflines_other": others,
        "ops_ms": {"factor_probe": round(probe_ms, 4), "factor_sparse": round(sparse_ms, 4),
                   "factor_redo": round(redo_ms, 4), "forward": round(fwd_ms, 4), "forward_levels_only": round(levels_ms, 4),
                   "logdet": round(ld_ms, 4), "inverse": round(inv_ms, 4),
                   "instrumented_step_ms": round((tp1 - tp0) * 1e3 / steps, 3)},
        "graph_build_s": round(graph_s, 2), "graph_phases_s": graph_phases,
        "graph_neighbour_search": "host" if args.host_knn else "device (graph_knn_device, incl. transfers)",
        "fused_forward": fused,
    }

    # ---- sampled check against the oracle at full size (outside the timed region)
    if not args.no_check:
        out["check"] = sampled_check(g, fac, v, xi, kern, w, n, k, n0)
    if not args.no_compare:
        # the plain FP64 path on the same points, graph and white noise
        v32, ld32 = v.double(), float(ld.item())
        del fac, dg, v
        torch.cuda.empty_cache()
        out["fp64_path_same_workload"] = compare_fp64(g, kern, xi_in, v32, ld32, args.steps, dev)
        del v32
        torch.cuda.empty_cache()
        out["k16_radial"] = k16_radial(args.steps, dev)
        out["matern_general_nu"] = matern_general(args.steps, dev)
        if args.workload == 3 and args.k is None:
            out["k16_same_distribution"] = same_distribution_k16(w, n, args.steps, dev, args.threads)
        out["adjoint_radial_2e22"] = adjoint_step(args.steps, dev)
    copy_gbs = copy_bandwidth(dev)
    out["copy_bandwidth_GBs"] = round(copy_gbs, 1)
    out["rooflines_other"]["forward+logdet"]["frac_of_copy"] = round(fl_gbs / copy_gbs, 4)
    if args.serve_requests > 0:
        out["serving"] = serving_run(args.serve_requests)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def fused_forward_run(dg, kern, xi, v_ref, ld_ref, steps, n):
    """Fused forward + logdet (vecchia_forward_fused): time per pass and its
    difference from the stored-factor step's v and logdet (same graph, same
    white noise); workspace bytes against the stored factor's."""
    import torch
    from paper_2606_11402_amd import FusedForward, workspace_bytes
    ff = FusedForward(dg, kern)
    vf = torch.empty_like(xi)
    ldf = torch.empty(1, dtype=torch.float64, device=xi.device)
    ff(xi, out=vf, logdet=ldf)
    ff.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ff(xi, out=vf, logdet=ldf)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    v_rel = float(((vf.double() - v_ref.double()).abs().max() / v_ref.double().abs().max()).item())
    ld_rel = abs(ldf.item() - ld_ref.item()) / abs(ld_ref.item())
    res = {"ms_per_pass": round(ms, 3), "points_per_s": n / (ms * 1e-3),
           "workspace_bytes": ff.workspace.numel(),
           "stored_factor_workspace_bytes": workspace_bytes(dg.n, dg.k, dg.n0, dg.precision),
           "v_rel_vs_stored_path": v_rel, "logdet_rel_vs_stored_path": ld_rel,
           "note": "Alg. 1 fused: per batch, each point rebuilds K_cc, factors it (double) and writes v_i; "
                   "no b or sigma stored; logdet from the same pass"}
    log("fused forward:", res)
    del ff, vf
    torch.cuda.empty_cache()
    return res


def copy_bandwidth(dev, nbytes=1 << 30, reps=10):
    """Device-to-device copy of 1 GiB (read + write), GB/s, HIP events."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def same_distribution_k16(w, n, steps, dev, threads):
    """The headline distribution and kernel at k = 16 (graph rebuilt)."""
    import torch
    from paper_2606_11402_amd import FP32, Factor, Graph, KernelParams
    from paper_2606_11402_amd import vecchia as vmod
    g = Graph(w.points(n), 16, w.n0, n_threads=threads, knn_device=str(dev))
    dg = g.to_device(FP32, dev)
    xi = torch.from_numpy(g.to_storage(w.xi(n))).float().to(dev)
    v = torch.empty(n, dtype=torch.float32, device=dev)
    ld = torch.empty(1, dtype=torch.float64, device=dev)
    fac = Factor(dg, KernelParams(w.kind, w.sigma, w.ell, w.nugget))
    ms = time_steps(fac, xi, v, ld, steps)
    vmod.profile_reset()
    vmod.profile_enable(True)
    for _ in range(steps):
        fac.forward(xi, out=v)
        fac.logdet(out=ld)
    prof = vmod.profile_read()
    vmod.profile_enable(False)
    fl_ms = sum(t for name, (t, _) in prof.items() if name.startswith("forward_") or name == "logdet") / steps
    bpp = apply_bytes_per_point(16, 4) + 4
    gbs = bpp * (n - w.n0) / (fl_ms * 1e-3) / 1e9
    res = {"k": 16, "ms_per_step": round(ms, 3), "points_per_s": n / (ms * 1e-3),
           "points_recomputed_fp64": fac.counts()[1], "forward+logdet_ms": round(fl_ms, 4),
           "forward+logdet_GBs": round(gbs, 1), "forward+logdet_frac": round(gbs / HBM_PEAK_GBS, 4),
           "levels": g.n_levels}
    log("k16 same distribution:", res)
    return res


def sweep_bytes(n, ns, k, esz):
    """Algorithmic bytes of the reverse sweep (w = (I - B)^-T vbar by batches,
    a gather over the children lists): per edge the packed child entry (4),
    its coefficient (esz) and the child's w (8, double); per point its two
    children offsets (8, each read once), vbar (esz), w written (8); per
    sparse point sigma (esz) and xibar written (esz)."""
    return ns * k * (12 + esz) + n * (16 + esz) + ns * 2 * esz


def theta_laneops_per_point(k, kind):
    """Algorithmic VALU lane-operations of the theta kernel for one sparse
    point: K_cc and its Cholesky again (the factor's count without the
    coefficient solve), the two solves of u = K_cc^-1 bbar (k^2), and the
    derivatives of the k(k+1)/2 distinct entries of K_cc and of the k
    entries of k_ci, each a kernel evaluation with its ell-derivative (about
    six operations more than the value alone) and two accumulations."""
    per_eval = {0: 12, 1: 16, 2: 11, 3: 18}[kind]
    factor = k * (k + 1) // 2 * per_eval + k ** 3 / 6.0 + k * k / 2.0 + 8 * k
    return factor + k * k + (k * (k + 1) // 2 + k) * (per_eval + 6 + 2)


def adjoint_step(steps, dev):
    """The gradient configuration (2^22 radial points, Matern-3/2, k = 16,
    FP32 path): factor + forward + logdet, then the reverse sweep and the
    theta kernel for loss = 1/2 |v - y|^2 / s^2 + logdet, s = 0.1.  The
    parts are timed with events on the library's stream: the backward with
    logdet_bar only runs the theta kernel (and the dense block) without the
    sweep, so the sweep's time is the difference of the two backward calls."""
    import torch
    import workloads
    from paper_2606_11402_amd import FP32, Factor, Graph, KernelParams
    w = workloads.WORKLOADS[4]
    g = Graph(w.points(w.n), w.k, w.n0)
    dg = g.to_device(FP32, dev, with_children=True)
    xi = torch.from_numpy(g.to_storage(w.xi(w.n))).float().to(dev)
    y = torch.from_numpy(g.to_storage(w.data(w.n))).float().to(dev)
    fac = Factor(dg, KernelParams(w.kind, w.sigma, w.ell, w.nugget))
    v = torch.empty_like(xi)
    scratch = None

    def step():
        nonlocal scratch
        fac.refactor()
        fac.forward(xi, out=v)
        vbar = (v - y) / 0.01
        _, _, theta = fac.backward(xi, v, v_bar=vbar, logdet_bar=1.0, scratch=scratch)
        return theta

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        theta = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps

    def timed(fn, reps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / reps

    vbar = (v - y) / 0.01
    reps = max(steps, 3)
    t_factor = timed(fac.refactor, reps)
    t_forward = timed(lambda: fac.forward(xi, out=v), reps)
    t_full = timed(lambda: fac.backward(xi, v, v_bar=vbar, logdet_bar=1.0, scratch=scratch), reps)
    t_theta = timed(lambda: fac.backward(xi, v, logdet_bar=1.0, scratch=scratch), reps)
    t_x = timed(lambda: fac.backward_x(xi, v, v_bar=vbar, logdet_bar=1.0), reps)
    t_sweep = max(t_full - t_theta, 1e-6)
    ns = w.n - w.n0
    sb = sweep_bytes(w.n, ns, w.k, 4)
    tl = theta_laneops_per_point(w.k, w.kind) * ns
    res = {"n": w.n, "k": w.k, "ms_per_step": round(ms, 3), "points_per_s": w.n / (ms * 1e-3),
           "step": "factor + forward + reverse sweep + theta kernel", "theta_bar": [float(t) for t in theta.cpu()],
           "parts_ms": {"factor": round(t_factor, 3), "forward": round(t_forward, 3),
                        "backward": round(t_full, 3), "theta_and_dense": round(t_theta, 3),
                        "sweep": round(t_sweep, 3),
                        "coordinates_backward_x": round(t_x, 3)},
           "levels": g.n_levels,
           "rooflines": {
               "sweep": {"bound": "hbm", "achieved": round(sb / (t_sweep * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(sb / (t_sweep * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "per_unit": "%.0f B per sparse point (k edges of 16 B, the point's own 28 B)" % (sb / ns),
                         "launches": g.n_levels + 1},
               "theta": {"bound": "alu", "achieved": round(tl / (t_theta * 1e-3) / 1e12, 3),
                         "peak": VALU_PEAK_TLANEOPS, "unit": "T lane-op/s",
                         "frac": round(tl / (t_theta * 1e-3) / 1e12 / VALU_PEAK_TLANEOPS, 4),
                         "per_unit": "%.0f lane-ops per sparse point" % (tl / ns),
                         "note": "time of the backward with logdet_bar only: theta kernel + dense block + reduction"}}}
    log("adjoint:", res)
    return res


def time_steps(fac, xi, v, ld, steps):
    import torch
    for _ in range(2):
        fac.refactor()
        fac.forward(xi, out=v)
        fac.logdet(out=ld)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fac.refactor()
        fac.forward(xi, out=v)
        fac.logdet(out=ld)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def compare_fp64(g, kern, xi_in, v32, ld32, steps, dev):
    """Plain FP64 path (FP64 storage and arithmetic throughout) on the same
    graph and white noise; the FP32 path's v and logdet against it."""
    import torch
    from paper_2606_11402_amd import FP64, Factor
    dg = g.to_device(FP64, dev)
    xi = torch.from_numpy(g.to_storage(xi_in)).double().to(dev)
    v = torch.empty(g.n, dtype=torch.float64, device=dev)
    ld = torch.empty(1, dtype=torch.float64, device=dev)
    fac = Factor(dg, kern)
    ms = time_steps(fac, xi, v, ld, steps)
    fac.status()
    ld64 = float(ld.item())
    v_rel = float(((v32 - v).abs().max() / v.abs().max()).item())
    log("fp64 path: %.3f ms/step" % ms)
    return {"ms_per_step": round(ms, 3), "points_per_s": g.n / (ms * 1e-3),
            "fp32_path_v_rel_err": v_rel, "fp32_path_logdet_rel_err": abs(ld32 - ld64) / abs(ld64),
            "note": "same points, graph and xi; errors of the FP32 path measured against this FP64 path"}


def k16_radial(steps, dev):
    """The k = 16 configuration (2^20 radial points, Matern-3/2, ell = 0.05):
    FP32 path and plain FP64 path, same graph and white noise."""
    import torch
    import workloads
    from paper_2606_11402_amd import FP32, FP64, Factor, Graph, KernelParams
    w = workloads.WORKLOADS[2]
    g = Graph(w.points(w.n), w.k, w.n0)
    kern = KernelParams(w.kind, w.sigma, w.ell, w.nugget)
    res, outs = {}, {}
    for prec, name in ((FP32, "fp32"), (FP64, "fp64")):
        dg = g.to_device(prec, dev)
        xi = torch.from_numpy(g.to_storage(w.xi(w.n))).to(dg.dtype).to(dev)
        v = torch.empty(g.n, dtype=dg.dtype, device=dev)
        ld = torch.empty(1, dtype=torch.float64, device=dev)
        fac = Factor(dg, kern)
        ms = time_steps(fac, xi, v, ld, steps)
        fac.status()
        res[name] = {"ms_per_step": round(ms, 3), "points_per_s": g.n / (ms * 1e-3),
                     "points_recomputed_fp64": fac.counts()[1]}
        outs[name] = (v.double(), float(ld.item()))
    v32, l32 = outs["fp32"]
    v64, l64 = outs["fp64"]
    res["fp32_vs_fp64"] = {"v_rel": float(((v32 - v64).abs().max() / v64.abs().max()).item()),
                           "logdet_rel": abs(l32 - l64) / abs(l64)}
    res["config"] = {"workload": w.name, "n": w.n, "k": w.k, "kernel": "M32", "ell": w.ell}
    log("k16 radial:", res)
    return res


def matern_general(steps, dev):
    """Cost of the general Matern kernel (kind 4, K_nu evaluated per entry)
    against the closed-form Matern-3/2 on the same graph: 2^20 uniform
    points, k = 16, ell = 0.02, FP64 path, factor + forward + logdet; and at
    nu = 3/2 the general kernel's results against the closed form's."""
    import torch
    import workloads
    from paper_2606_11402_amd import FP64, M32, MATERN, Factor, Graph, KernelParams
    n, k, n0 = 1 << 20, 16, 128
    g = Graph(workloads.uniform(n, 2026), k, n0, knn_device=dev)
    dg = g.to_device(FP64, dev)
    xi = torch.from_numpy(g.to_storage(workloads.white_noise(n, 2126))).to(dg.dtype).to(dev)
    res, outs = {"config": {"workload": "uniform-2^20-k16-fp64", "n": n, "k": k, "ell": 0.02}}, {}
    for name, kern in (("m32", KernelParams(M32, 1.0, 0.02)), ("matern_nu_1.5", KernelParams(MATERN, 1.0, 0.02, 0.0, 1.5)),
                       ("matern_nu_1.7", KernelParams(MATERN, 1.0, 0.02, 0.0, 1.7))):
        v = torch.empty(n, dtype=dg.dtype, device=dev)
        ld = torch.empty(1, dtype=torch.float64, device=dev)
        fac = Factor(dg, kern)
        ms = time_steps(fac, xi, v, ld, steps)
        fac.status()
        res[name] = {"ms_per_step": round(ms, 3), "points_per_s": n / (ms * 1e-3)}
        outs[name] = (v.clone(), float(ld.item()))
        del fac
    (va, la), (vb, lb) = outs["matern_nu_1.5"], outs["m32"]
    res["nu_1.5_vs_m32"] = {"v_rel": float(((va - vb).abs().max() / vb.abs().max()).item()),
                            "logdet_rel": abs(la - lb) / abs(lb)}
    log("general Matern:", res)
    return res


def serving_run(n_requests):
    """A prefix of the serving request stream (N log-uniform in [1e3, 1e6],
    k in {8, 16, 32}, ell ~ U(0.01, 0.2), forward / inverse / logdet, FP32):
    closed-loop capacity, then Poisson arrivals at 0.7 of it.  Graphs of at
    least 2^15 points are built on the GPU (3 GiB of slices for the 14
    graph workers), smaller ones on the host."""
    import workloads
    from paper_2606_11402_amd.serve import Server, run_stream
    reqs = workloads.request_stream(n_requests, rate=1.0)
    budget = 8 << 30
    gdev = 3 << 30
    srv = Server(budget, n_streams=8, graph_workers=14, graph_device_bytes=gdev)
    closed = run_stream(reqs, srv, rate=None)
    graphs_on_device = srv.stats()["graphs_on_device"]
    srv.close()
    srv = Server(budget, n_streams=8, graph_workers=14, graph_device_bytes=gdev)
    lam = 0.7 * closed["req_per_s"]
    opened = run_stream(reqs, srv, rate=lam)
    srv.close()
    keep = ("req_per_s", "points_per_s", "latency_p50_s", "latency_p99_s", "graph_p50_s", "graph_p99_s",
            "queue_p50_s", "device_p50_s", "device_p99_s", "peak_hbm_bytes")
    log("serving: capacity %.1f req/s, p50 %.3fs p99 %.3fs at 0.7x" % (closed["req_per_s"], opened["latency_p50_s"],
                                                                     opened["latency_p99_s"]))
    return {"requests": n_requests, "hbm_budget_bytes": budget, "graph_device_bytes": gdev,
            "graphs_on_device_closed_loop": graphs_on_device, "closed_loop": {a: closed[a] for a in keep},
            "open_loop_0.7": dict({a: opened[a] for a in keep}, lambda_req_per_s=lam)}


def sampled_check(g, fac, v, xi, kern, w, n, k, n0, samples=256):
    """Per-point checks the oracle can do one by one at any N: b and sigma of
    sampled points from Eq. (2) in FP64, and the forward identity
    v_i = b_i . v[c(i)] + sigma_i xi_i evaluated with the oracle's b, sigma on
    the GPU's own v."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(12345)
    rows = rng.choice(g.ns, size=min(samples, g.ns), replace=False)
    xs = g.points()                                    # FP64 values of the FP32 coordinates
    nb = g.nbr(0)[rows]
    b_gpu, s_gpu = fac.coefficient_rows(rows)
    b_gpu = g.to_row_order(b_gpu, rows)                # device rows -> the rows of nbr(0)
    vh = v.double().cpu().numpy()
    xih = xi.double().cpu().numpy()
    ok_kern = oracle.Kernel(kern.kind, kern.sigma, kern.ell, kern.nugget)
    eb = es = ev = 0.0
    bmax = smax = vmax = 0.0
    for t, r in enumerate(rows):
        c = nb[t][nb[t] >= 0]
        b, s = oracle.conditional(xs[c], xs[n0 + r], ok_kern)
        eb = max(eb, float(np.max(np.abs(b_gpu[t][:len(c)] - b))))
        bmax = max(bmax, float(np.max(np.abs(b))))
        es = max(es, abs(float(s_gpu[t]) - s))
        smax = max(smax, s)
        vi = float(b @ vh[c]) + s * float(xih[n0 + r])
        ev = max(ev, abs(vh[n0 + r] - vi))
        vmax = max(vmax, abs(vi))
    return {"samples": int(len(rows)), "b_rel": float(eb / bmax), "sigma_rel": float(es / smax),
            "forward_identity_rel": float(ev / vmax), "logdet": float(fac.logdet().item())}


_CPU_STATE = None   # (oracle graph, kernel) inherited by the forked baseline workers


def _cpu_worker_init():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)            # one BLAS thread per worker process
    except Exception:
        pass


def _cpu_factor_rows(rows):
    import oracle
    og, kern = _CPU_STATE
    fac = oracle.factor(og, kern, rows=rows)
    return fac.b, fac.sigma


def cpu_baseline(w, k, n0, n_sample, passes):
    """The FP64 oracle (as written, not tuned) on a sample of the same
    workload: factor + forward + logdet, the oracle's own graph built untimed.
    Multi-core: the sparse rows of the factor are split over a pool of forked
    worker processes (one per core of the host's share, one BLAS thread each);
    the forward (batch after batch) and the logdet run in the parent.  The
    oracle's work per point does not depend on N (the factor is per point, the
    forward one vectorised pass per batch), so points/s of the sample stands
    for the full workload.  The single-core rate is measured beside it."""
    import concurrent.futures
    import multiprocessing
    import numpy as np
    import oracle
    import workloads
    global _CPU_STATE
    gen = {"uniform": workloads.uniform, "radial": workloads.radial, "clumped": workloads.clumped,
           "gaussian": workloads.gaussian}[w.dist]
    x = workloads.as_fp32_exact(gen(n_sample, w.number))
    log("cpu baseline: oracle graph for N=%d (untimed)" % n_sample)
    og = oracle.build_graph(x, k, n0)
    kern = oracle.Kernel(w.kind, w.sigma, w.ell, w.nugget)
    xi = workloads.white_noise(n_sample, w.number + 100)[og.perm]
    _CPU_STATE = (og, kern)
    ns = n_sample - n0
    cores = max(1, min(16, os.cpu_count() or 1))       # the host's CPU share on the GPU machine
    chunks = np.array_split(np.arange(ns), cores * 4)

    def one_pass(pool):
        if pool is None:
            fac = oracle.factor(og, kern)
        else:
            parts = list(pool.map(_cpu_factor_rows, chunks))
            fac = oracle.Factor(oracle.vecchia.dense_block(og.xs, n0, kern),
                                np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]))
        oracle.forward(og, fac, xi)
        return oracle.logdet(fac)

    ctx = multiprocessing.get_context("fork")
    with concurrent.futures.ProcessPoolExecutor(cores, mp_context=ctx, initializer=_cpu_worker_init) as pool:
        ld_multi = one_pass(pool)                       # warm the workers
        t = time.perf_counter()
        for _ in range(passes):
            one_pass(pool)
        dt_multi = time.perf_counter() - t
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            t = time.perf_counter()
            ld_single = one_pass(None)
            dt_single = time.perf_counter() - t
    except ImportError:
        t = time.perf_counter()
        ld_single = one_pass(None)
        dt_single = time.perf_counter() - t
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    res = {"value": passes * n_sample / dt_multi, "unit": "points/s", "cores": cores, "kind": "oracle",
           "sample": "same distribution, kernel and k at N=%d (the oracle's brute-force graph, built untimed, is "
                     "quadratic in N); %d passes of factor+forward+logdet, FP64 NumPy, factor rows over %d "
                     "worker processes with one BLAS thread each; per-point work is independent of N, so the "
                     "rate stands for the full workload" % (n_sample, passes, cores),
           "seconds": round(dt_multi, 2), "single_core_points_per_s": n_sample / dt_single,
           "single_core_seconds": round(dt_single, 2), "logdet_multi_equals_single": ld_multi == ld_single,
           "host_cpu": cpu, "host_threads_visible": os.cpu_count()}
    log("cpu baseline:", res)
    return res


if __name__ == "__main__":
    main()
