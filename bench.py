"""Benchmark: time to relative residual 1e-10 on the 256^3 variable-coefficient
problem (64 boxes of 64^3, Dirichlet walls, lognormal b with sigma 1, uniform
rhs), FP64 V-cycles and FP32 V-cycles inside FP64 refinement, on one GPU.

One step = four solves from phi = 0 on the same device-resident input: FP64
V-cycles, the FP32 V-cycle inside FP64 refinement, and conjugate gradients
preconditioned by one symmetric V-cycle in FP64 and in FP32.  The JSON line
reports the FP64 V-cycle time as `value`, every variant's time, the level-0
smoother's achieved bandwidth (algorithmic bytes / mean launch duration from
HIP events on the solver's stream), the library's own streaming copy as the
achievable rate, and the CPU oracle's whole solve of the same problem, timed
on the host, whose solution gives each variant's error.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to 1e-10 rel residual, 256^3 var-coef (FP64 vs FP32+refine); smoother GB/s"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--profile-steps", type=int, default=2,
                   help="extra solves after the timed ones with per-kernel HIP events")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--tune", type=int, default=2, help="0 default tiles, 1 cache, 2 search")
    p.add_argument("--aggregate", type=int, default=1)
    p.add_argument("--fused-min-edge", type=int, default=0,
                   help="fused red/black sweeps on levels whose boxes are all this large (0 = off)")
    p.add_argument("--smoother-shape", default=None,
                   help="lx,ly,tz,unroll[,whole_pairs]: level-0 half-sweep tile shape applied "
                        "after tuning (counter runs per shape)")
    p.add_argument("--f32-smoother-shape", default=None,
                   help="lx,ly,tz,unroll[,mapping]: the same for the FP32 V-cycle solvers only "
                        "(after --smoother-shape); mapping 1 = whole x-pairs, 2 = one x-quad per lane")
    p.add_argument("--cell-shape", default=None,
                   help="lx,ly,tz,unroll: level-0 tiles of the residual kernels (the stop test, "
                        "the FP64 residual of the FP32 cycle), applied after tuning (counter runs)")
    p.add_argument("--rr-shape", default=None,
                   help="lx,ly,tz: level-0 tiles of the residual pass restricting into level 1, "
                        "applied after tuning (counter runs)")
    p.add_argument("--trace-solve", action="store_true",
                   help="only the FP64 V-cycle solver of the 256^3 workload: set-up (tuned), three "
                        "warm-up solves and one more, no JSON line (a kernel trace of one tuned "
                        "solve, the last one in the trace)")
    p.add_argument("--quiet", action="store_true")
    p.add_argument("--workload", default="c1", choices=["c1", "c2", "c3", "c4", "nodal"],
                   help="c1: the headline 256^3 line; c2: 512^3 uneven boxes, four variants; "
                        "c3: 128^3 adjoint gradient; c4: two-level composite (supplementary); "
                        "nodal: 256^3 nodal finite-element solve")
    return p.parse_args()


ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_gsrb_abec256_lognormal_64boxes.md")


def kernel_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "tables.hpp"):
        with open(os.path.join(ROOT, "paper_2009_12009_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _classes_key(classes):
    """{x extent: (lx, ly, tz)} -> the canonical text of a block's `classes:` line."""
    return "; ".join(f"{int(x)} {v[0]} {v[1]} {v[2]}"
                     for x, v in sorted((int(x), v) for x, v in (classes or {}).items()))


def measured_traffic(kernel, shape, classes=None):
    """HBM bytes per launch of the level-0 half-sweep from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or
    None when the summary is missing, was taken on other kernel sources, or holds
    no block for this kernel, launch shape and per-class tile table (a block
    without a `classes:` line is the uniform table)."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    # fenced blocks alternate with prose: the odd pieces are the blocks
    for block in text.split("```")[1::2]:
        kv = {}
        for line in block.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        try:
            if (kv.get("source_sha256") != kernel_source_sha256() or kv.get("kernel") != kernel
                    or tuple(int(x) for x in kv["shape"].split()) != tuple(shape)
                    or kv.get("classes", "") != _classes_key(classes)):
                continue
            return (float(kv["fetch_kib_per_dispatch"]) * 1024 * float(kv["fetch_scale"])
                    + float(kv["write_kib_per_dispatch"]) * 1024 * float(kv["write_scale"]))
        except (KeyError, ValueError):
            continue
    return None


def log(msg, quiet=False):
    if not quiet:
        print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU layout is "
              "a design, not a build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2009_12009_amd as P
    import workloads as W

    torch.cuda.set_device(0)
    q = args.quiet
    if args.workload == "c2":
        return bench_c2(args)
    if args.workload == "c3":
        return bench_c3(args)
    if args.workload == "nodal":
        return bench_nodal(args)
    if args.workload == "c4":
        return bench_c4(args)
    t0 = time.perf_counter()
    cfg = W.config_c1()
    n, boxes = cfg["n"], cfg["boxes"]
    dom = W.domain_box(n)
    f_boxes = W.scatter_cells(cfg["rhs"], boxes)
    rhs = P.MultiFab.from_numpy(boxes, f_boxes, 0)
    bmf = []
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        bmf.append(P.MultiFab.from_numpy(boxes, W.scatter_faces(cfg["faces"][d], boxes, d), 0,
                                         ixtype=tuple(e)))
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s", q)

    common = dict(tune=args.tune, aggregate=args.aggregate, fused_min_edge=args.fused_min_edge)
    if args.trace_solve:
        s = P.MLMG(boxes, dom, cfg["periodic"], 1.0, 1.0, b=bmf, opts=dict(precision=0, **common))
        phi = s.cell_mf(1, fill=0.0)
        for k in range(5):
            phi.data.zero_()
            info = s.solve(phi, rhs, 1e-10)
            log(f"solve {k}: {info['iters']} cycles, {info['solve_ms']:.2f} ms", q)
        torch.cuda.synchronize()
        s.close()
        return
    solvers = {
        "f64": P.MLMG(boxes, dom, cfg["periodic"], 1.0, 1.0, b=bmf, opts=dict(precision=0, **common)),
        "f32_refine": P.MLMG(boxes, dom, cfg["periodic"], 1.0, 1.0, b=bmf,
                             opts=dict(precision=1, **common)),
        # conjugate gradients preconditioned by one symmetric V-cycle per iteration
        "f64_mgpcg": P.MLMG(boxes, dom, cfg["periodic"], 1.0, 1.0, b=bmf,
                            opts=dict(precision=0, krylov=1, **common)),
        # the same with the V-cycle in FP32 (CG in FP64)
        "f32_mgpcg": P.MLMG(boxes, dom, cfg["periodic"], 1.0, 1.0, b=bmf,
                            opts=dict(precision=1, krylov=1, **common)),
    }
    if args.smoother_shape:
        v = [int(x) for x in args.smoother_shape.split(",")]
        kern = 2 if len(v) == 5 and v[4] else 0
        for s in solvers.values():
            s.set_tile_shape(kern, *v[:4])
    if args.f32_smoother_shape:
        v = [int(x) for x in args.f32_smoother_shape.split(",")]
        kern = {0: 0, 1: 2, 2: 5}[v[4] if len(v) == 5 else 0]
        for k in ("f32_refine", "f32_mgpcg"):
            solvers[k].set_tile_shape(kern, *v[:4])
    if args.cell_shape:
        v = [int(x) for x in args.cell_shape.split(",")]
        for s in solvers.values():
            s.set_tile_shape(1, *v[:4])
    if args.rr_shape:
        v = [int(x) for x in args.rr_shape.split(",")]
        for s in solvers.values():
            s.set_tile_shape(4, *v[:3])
    phis = {k: s.cell_mf(1, fill=0.0) for k, s in solvers.items()}
    setup_ms = {k: s.solve(phis[k], rhs, 1e-10)["setup_ms"] for k, s in solvers.items()}

    def step(record):
        out = {}
        for k, s in solvers.items():
            phis[k].data.zero_()
            info = s.solve(phis[k], rhs, 1e-10)
            assert info["converged"], (k, info)
            out[k] = info
            if record is not None:
                record[k].append(info)
        return out

    for _ in range(args.warmup):
        step(None)
    rec = {k: [] for k in solvers}
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t1) * 1e3
    ms_step = wall / args.steps

    # kernel durations: HIP events around every level-0 launch, recorded in
    # extra solves after the timed region (the event records add gaps, so the
    # timed solves run without them)
    for s in solvers.values():
        s.profile(True)
    for _ in range(args.profile_steps):
        step(None)
    torch.cuda.synchronize()

    # level-0 smoother: mean launch duration over the profiled solves
    ncell = n ** 3
    gs = {}
    for k, s in solvers.items():
        tot, cnt = s.kernel_stats(P._lib.FAM_SMOOTH)
        word = 4 if k.startswith("f32") else 8
        mean_ms = tot / max(cnt, 1)
        alg_bytes = 6 * word * ncell  # phi in, phi out, f, b_x, b_y, b_z
        gs[k] = dict(mean_ms=mean_ms, launches=cnt, bytes=alg_bytes,
                     gbps=alg_bytes / (mean_ms * 1e-3) / 1e9 if cnt else None)
        fam = {}
        for name, fid in (("smooth", 0), ("residual", 1), ("exchange", 2), ("restrict", 3),
                          ("prolong", 4), ("coarse_levels", 5), ("update", 6), ("rim", 7)):
            t, c = s.kernel_stats(fid)
            fam[name] = dict(ms_per_solve=t / max(args.profile_steps, 1),
                             launches_per_solve=c / max(args.profile_steps, 1))
        gs[k]["families"] = fam
        # rim launches only come with fused sweeps (the tuner may have kept half-sweeps)
        gs[k]["fused"] = fam["rim"]["launches_per_solve"] > 0
        gs[k]["tile_shapes"] = {"smoother": s.tile_shape(0), "cell": s.tile_shape(1),
                                "fused_sweep": s.tile_shape(3),
                                "resid_restrict": s.tile_shape(4),
                                "smoother_classes": {str(x): list(v) for x, v in
                                                     sorted(s.class_tile_shapes().items())}}
        s.profile(False)

    # every variant's last solution, for its error against the oracle's (taken before
    # the stand-alone smoother timing below sweeps the FP64 solver's phi in place)
    sols = {k: W.gather_cells(phis[k].valid_numpy(), boxes, n) for k in solvers}

    # the level-0 FP64 half-sweep launched alone, without ghost write-through
    ms_alone = solvers["f64"].time_smoother(phis["f64"], rhs, reps=20)
    smoother_alone = {"mean_ms": ms_alone, "gbps": 6 * 8 * ncell / (ms_alone * 1e-3) / 1e9}

    # the library's streaming copy (one 16-byte element per lane) over 1 GiB
    # as the achievable rate; launched on torch's current stream, which the
    # events are recorded on
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        P.stream_copy(dst, src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        P.stream_copy(dst, src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * src.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    assert bool(torch.all(dst == 1.0))
    del src, dst

    t64 = [r["solve_ms"] for r in rec["f64"]]
    t32 = [r["solve_ms"] for r in rec["f32_refine"]]
    tpcg = [r["solve_ms"] for r in rec["f64_mgpcg"]]
    tpcg32 = [r["solve_ms"] for r in rec["f32_mgpcg"]]
    result = {
        "metric": METRIC,
        "value": float(np.median(t64)),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n": n, "boxes": len(boxes), "box_edge": 64,
                   "bc": "dirichlet0", "alpha": 1.0, "beta": 1.0, "b": "exp(N(0,1)) seed 1, "
                   "harmonic faces", "rhs": "U[-1,1] seed 2", "rel_tol": 1e-10,
                   "nu1": 2, "nu2": 2, "levels": rec["f64"][0]["nlevels"],
                   "bottom": "CG rel 1e-4", "tune": args.tune, "aggregate": args.aggregate,
                   "fused_min_edge": args.fused_min_edge},
        "time_to_tol_ms": {"f64": float(np.median(t64)), "f32_refine": float(np.median(t32)),
                           "f64_mgpcg": float(np.median(tpcg)),
                           "f32_mgpcg": float(np.median(tpcg32))},
        "cycles": {k: rec[k][0]["iters"] for k in rec},
        "final_rel_resid": {k: rec[k][-1]["rel_resid"] for k in rec},
        "setup_ms": setup_ms,
        "profiled_solves": args.profile_steps,
        "smoother": {k: {kk: v for kk, v in g.items() if kk != "families"} for k, g in gs.items()},
        "time_by_family_ms": {k: g["families"] for k, g in gs.items()},
        "tile_shapes": {k: g["tile_shapes"] for k, g in gs.items()},
        "copy_kernel_gbps": copy_gbps,
        "copy_kernel": "k_stream_copy (mg_stream_copy), 1 GiB, 16 B per lane",
        "smoother_alone_f64": smoother_alone,
    }
    g64 = gs["f64"]
    kname = ("k_sweep<double> level 0, one fused red+black sweep (64 boxes of 64^3)"
             if g64["fused"] else
             "k_gsrb<double> level 0, one half-sweep with face-ghost write-through "
             "(64 boxes of 64^3)")
    traffic = None if g64["fused"] else measured_traffic(
        "k_gsrb<double>", g64["tile_shapes"]["smoother"], g64["tile_shapes"]["smoother_classes"])
    result["roofline"] = {
        "bound": "hbm",
        "achieved": g64["gbps"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": g64["gbps"] / HBM_PEAK_GBS if g64["gbps"] else None,
        "traffic": traffic,
        "kernel": kname,
        "alg_bytes_per_launch": g64["bytes"],
        "mean_launch_ms": g64["mean_ms"],
    }

    if not args.no_cpu:
        base, ophi = cpu_baseline(cfg, f_boxes, args, q)
        result["cpu_baseline"] = base
        # the oracle stops at the same test (max-norm 1e-10); its cycle count
        # must equal the FP64 V-cycle solve's
        result["rel_l2_vs_oracle"] = {k: float(np.linalg.norm(v - ophi) / np.linalg.norm(ophi))
                                      for k, v in sols.items()}
        result["oracle_cycles"] = base["cycles"]
    print(json.dumps(result), flush=True)
    for s in solvers.values():
        s.close()


def _face_mfs(P, W, cfg, boxes):
    out = []
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        out.append(P.MultiFab.from_numpy(boxes, W.scatter_faces(cfg["faces"][d], boxes, d), 0,
                                         ixtype=tuple(e)))
    return out


def bench_c2(args):
    """512^3 guillotine boxes: {FP64, FP32+refine} x {graph + tuned tiles, plain launches with
    default tiles}, time to 1e-10 from phi = 0 (median of the timed solves)."""
    import numpy as np
    import torch

    import paper_2009_12009_amd as P
    import workloads as W

    t0 = time.perf_counter()
    cfg = W.config_c2()
    n, boxes = cfg["n"], cfg["boxes"]
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_cells(cfg["rhs"], boxes), 0)
    bmf = _face_mfs(P, W, cfg, boxes)
    del cfg["rhs"], cfg["bcell"]
    log(f"c2 inputs ({len(boxes)} boxes) in {time.perf_counter() - t0:.1f} s", args.quiet)
    edges = {}
    for b in boxes:
        for d in range(3):
            e = b[1][d] - b[0][d] + 1
            edges[e] = edges.get(e, 0) + 1
    out = {"metric": "time to 1e-10 rel residual, 512^3 uneven boxes", "unit": "ms",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "config": {"workload": "abec512_guillotine", "boxes": len(boxes), "edge_histogram": edges,
                      "aggregate": args.aggregate}, "variants": {}}
    phi = P.MultiFab(boxes, 1, fill=0.0)
    # graph replay and tuning measured apart: tuned tiles (per box class where
    # that wins) and default tiles at equal graph setting, then plain launches
    for prec in (0, 1):
        for graph, tune, tag in ((1, 2, "graph_tuned"), (1, 0, "graph_default"),
                                 (0, 0, "plain_default")):
            name = f"{'f64' if prec == 0 else 'f32_refine'}_{tag}"
            s = P.MLMG(boxes, W.domain_box(n), cfg["periodic"], 1.0, 1.0, b=bmf,
                       opts=dict(precision=prec, use_graph=graph, tune=tune,
                                 aggregate=args.aggregate))
            times = []
            for k in range(args.warmup + args.steps):
                phi.data.zero_()
                info = s.solve(phi, rhs, 1e-10)
                assert info["converged"], info
                if k >= args.warmup:
                    times.append(info["solve_ms"])
            out["variants"][name] = {"time_to_tol_ms": float(np.median(times)),
                                     "cycles": info["iters"], "levels": info["nlevels"],
                                     "rel_resid": info["rel_resid"], "setup_ms": info["setup_ms"],
                                     "smoother_shape": s.tile_shape(0),
                                     "smoother_class_shapes": {str(k): list(v) for k, v in
                                                               s.class_tile_shapes().items()}}
            log(f"{name}: {np.median(times):.1f} ms, {info['iters']} cycles", args.quiet)
            s.close()
            torch.cuda.synchronize()
    out["value"] = out["variants"]["f64_graph_tuned"]["time_to_tol_ms"]
    print(json.dumps(out), flush=True)


def bench_c3(args):
    """128^3, 8 boxes of 64^3, sigma 0.5: forward solve, backward (adjoint solve + face
    gradient), and the face-gradient kernel's bandwidth."""
    import numpy as np
    import torch

    import paper_2009_12009_amd as P
    import workloads as W

    cfg = W.config_c3()
    n, boxes = cfg["n"], cfg["boxes"]
    s = P.MLMG(boxes, W.domain_box(n), cfg["periodic"], 1.0, 1.0,
               opts=dict(tune=2, aggregate=args.aggregate))
    f = torch.from_numpy(np.concatenate([x.ravel(order="F") for x in
                                         W.scatter_cells(cfg["rhs"], boxes)])).cuda()
    logb = [torch.from_numpy(P.global_to_xfast(np.log(cfg["faces"][d]))).cuda() for d in range(3)]
    logbt = [torch.from_numpy(P.global_to_xfast(np.log(cfg["faces_target"][d]))).cuda()
             for d in range(3)]
    with torch.no_grad():
        phi_t = P.mg_solve(f, *logbt, s, 1e-10)
    fw, bw = [], []
    for k in range(args.warmup + args.steps):
        fr = f.clone().requires_grad_(True)
        lb = [x.clone().requires_grad_(True) for x in logb]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi = P.mg_solve(fr, *lb, s, 1e-10)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = 0.5 * torch.sum((phi - phi_t) ** 2)
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if k >= args.warmup:
            fw.append((t1 - t0) * 1e3)
            bw.append((t2 - t1) * 1e3)
    # face-gradient kernel alone
    ph = P.MultiFab(boxes, 1, fill=0.5)
    lm = P.MultiFab(boxes, 1, fill=0.25)
    for _ in range(2):
        s.face_grad_logb_global(ph, lm)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    # HIP events around the kernel itself on the solver's stream (profile family 8)
    s.profile(True)
    e0.record()
    for _ in range(reps):
        s.face_grad_logb_global(ph, lm)
    e1.record()
    torch.cuda.synchronize()
    t_k, n_k = s.kernel_stats(8)
    s.profile(False)
    ms = t_k / max(n_k, 1)
    # the whole call: ghost exchange of phi and lambda, output allocation, the kernel
    ms_call = e0.elapsed_time(e1) / reps
    nf = 3 * (n + 1) * n * n
    # what the method must move: per face b in and the gradient out, per cell phi and lambda
    # once (one pass over all three directions)
    alg = nf * 8 * 2 + 2 * n ** 3 * 8
    out = {"metric": "adjoint gradient, 128^3 (8 boxes of 64^3)", "unit": "ms", "n_gpus": 1,
           "higher_is_better": False, "data": "synthetic",
           "config": {"workload": "adjoint128", "sigma": 0.5, "rel_tol": 1e-10},
           "value": float(np.median(fw) + np.median(bw)),
           "forward_ms": float(np.median(fw)), "backward_ms": float(np.median(bw)),
           "face_grad_ms": ms, "face_grad_gbps": alg / (ms * 1e-3) / 1e9,
           "face_grad_alg_bytes": alg, "face_grad_call_ms": ms_call,
           "face_grad_timing": "kernel alone: HIP events on the solver's stream; call: "
                               "exchange of phi and lambda, output allocation and the kernel"}
    print(json.dumps(out), flush=True)
    s.close()


def bench_c4(args):
    """Two-level composite: 256^3 coarse in 64 boxes, fine boxes over the cells
    where the 4-blob rhs exceeds half its maximum; FP64 to composite 1e-10."""
    import numpy as np
    import torch

    import paper_2009_12009_amd as P
    import workloads as W
    from workloads import amr

    t0 = time.perf_counter()
    cfg = amr.config_c4()
    cb, fb = cfg["boxes"], cfg["fine_boxes"]
    bcm = _face_mfs(P, W, cfg, cb)
    bfm = []
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        bfm.append(P.MultiFab.from_numpy(fb, amr.fine_faces(cfg["bcell"], cfg["faces"], fb, d), 0,
                                         ixtype=tuple(e)))
    rc = P.MultiFab.from_numpy(cb, W.scatter_cells(cfg["rhs"], cb), 0)
    rf = P.MultiFab.from_numpy(fb, amr.fine_rhs(fb, cfg["centres"], 2 * cfg["n"]), 0)
    log(f"c4 inputs ({len(fb)} fine boxes) in {time.perf_counter() - t0:.1f} s", args.quiet)
    res = {}
    for name, prec, kry in (("f64", 0, 0), ("f32_refine", 1, 0), ("f64_fgmres", 0, 1),
                            ("f32_fgmres", 1, 1)):
        s = P.CompositeMLMG(cb, fb, W.domain_box(cfg["n"]), 1.0, 1.0, b_c=bcm, b_f=bfm,
                            opts=dict(tune=2, aggregate=args.aggregate, precision=prec,
                                      krylov=kry))
        pc = s.coarse_mf(1, fill=0.0)
        pf = s.fine_mf(1, fill=0.0)
        times = []
        for k in range(args.warmup + args.steps):
            pc.data.zero_()
            pf.data.zero_()
            info = s.solve(pc, pf, rc, rf, 1e-10)
            assert info["converged"], info
            if k >= args.warmup:
                times.append(info["solve_ms"])
        res[name] = dict(time_to_tol_ms=float(np.median(times)), cycles=info["iters"],
                         rel_resid=info["rel_resid"], setup_ms=info["setup_ms"])
        s.close()
    fine_cells = sum(int(np.prod([h - l + 1 for l, h in zip(*b)])) for b in fb)
    out = {"metric": "time to 1e-10 composite rel residual, two-level 256^3 + blob refinement",
           "unit": "ms", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "dtype": "f64", "value": res["f64"]["time_to_tol_ms"],
           "config": {"workload": "composite256", "fine_boxes": len(fb), "fine_cells": fine_cells,
                      "aggregate": args.aggregate},
           "variants": res}
    print(json.dumps(out), flush=True)
    torch.cuda.synchronize()


def bench_nodal(args):
    """256^3 cells (64 boxes of 64^3), Dirichlet walls, nodal -div(sigma grad phi) = f with
    cell sigma = exp(N(0,1)) (seed 1) and f ~ U[-1,1] on the nodes (seed 2): time to a max-norm
    relative residual of 1e-10 from phi = 0, and the finest-level Jacobi sweep's bandwidth."""
    import numpy as np
    import torch

    import paper_2009_12009_amd as P
    import workloads as W

    n = 256
    cfg = W.config_nodal(n, 64)
    boxes, per = cfg["boxes"], cfg["periodic"]
    sig = P.MultiFab.from_numpy(boxes, W.scatter_cells(cfg["sigma_cells"], boxes), 0)
    G = W.nodes_from_unknowns(cfg["rhs_unknowns"], n, per)
    rhs = P.MultiFab.from_numpy(boxes, W.scatter_nodes(G, boxes, 0), 0, ixtype=(1, 1, 1))
    del G
    variants = {}
    for name, kry in (("vcycle", 0), ("mgpcg", 1)):
        sv = P.NodalMLMG(boxes, W.domain_box(n), per, sigma=sig,
                         opts=dict(min_bottom_edge=4, krylov=kry, tune=2))
        phi = sv.node_mf(0, fill=0.0)
        tv = []
        for k in range(args.warmup + args.steps):
            phi.data.zero_()
            torch.cuda.synchronize()
            iv = sv.solve(phi, rhs, 1e-10)
            assert iv["converged"], iv
            if k >= args.warmup:
                tv.append(iv["solve_ms"])
        variants[name] = {"time_to_tol_ms": float(np.median(tv)), "iterations": iv["iters"],
                          "final_rel_resid": iv["rel_resid"]}
        if kry == 0:
            s, info, times = sv, iv, tv
        else:
            sv.close()
    m = W.nodal_unknown_shape(n, per)
    nodes = m[0] * m[1] * m[2]
    ms_sweep = s.time_smoother(20)
    # per unknown node: phi in, phi out, f, and one cell coefficient (the (m+1)^3 sigma array)
    alg = 8 * (3 * nodes + (m[0] + 1) * (m[1] + 1) * (m[2] + 1))
    gbps = alg / (ms_sweep * 1e-3) / 1e9
    out = {"metric": "time to 1e-10 rel residual, nodal 256^3 var-coef (FP64)", "unit": "ms",
           "value": float(np.median(times)), "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": False, "dtype": "f64",
           "data": "synthetic", "vs_baseline": None,
           "config": {"workload": "nodal256_lognormal_64boxes", "n": n, "boxes": len(boxes),
                      "bc": "dirichlet0", "sigma": "exp(N(0,1)) per cell, seed 1",
                      "rhs": "U[-1,1] per unknown node, seed 2", "rel_tol": 1e-10,
                      "nu1": 2, "nu2": 2, "jacobi_weight": 1.0, "levels": info["nlevels"],
                      "bottom": "CG rel 1e-4"},
           "time_to_tol_ms": {k: v["time_to_tol_ms"] for k, v in variants.items()},
           "iterations": {k: v["iterations"] for k, v in variants.items()},
           "variants": "vcycle: V-cycles (value); mgpcg: CG preconditioned by one V-cycle",
           "cycles": info["iters"], "ms_per_cycle": float(np.median(times)) / info["iters"],
           "final_rel_resid": info["rel_resid"], "setup_ms": info["setup_ms"],
           "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbps / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "k_nd_sweep0 (finest-level Jacobi sweep, 255^3 nodes)",
                        "alg_bytes_per_launch": alg, "mean_launch_ms": ms_sweep}}
    s.close()
    if not args.no_cpu:
        import oracle.nodal as ON
        nc = 64
        c64 = W.config_nodal(nc, nc)
        t0 = time.perf_counter()
        c0 = time.process_time()
        _, oinfo = ON.nodal_solve(c64["sigma_cells"], c64["periodic"], c64["rhs_unknowns"], 1e-10,
                                  opts=ON.NodalOpts(min_bottom_cells=4))
        wall = time.perf_counter() - t0
        cpu = time.process_time() - c0
        scale = (nodes / float((nc - 1) ** 3)) * (info["iters"] / float(oinfo["iters"]))
        out["cpu_baseline"] = {
            "value": wall * 1e3 * scale, "unit": "ms", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": f"whole oracle solve of the same generator at {nc}^3 ({oinfo['iters']} cycles, "
                      f"{wall:.1f} s), scaled by the unknown-node ratio and the cycle ratio",
            "sample_seconds": wall}
    print(json.dumps(out), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, f_boxes, args, q):
    """The oracle as it stands, on the host: one whole oracle.solve of the same
    256^3 problem from phi = 0 to max-norm 1e-10 (the same aggregated
    hierarchy, smoother and bottom tolerance as the GPU's FP64 V-cycles),
    timed with perf_counter around the solve only (its hierarchy is built
    beforehand, as mg_create builds the GPU's).  Returns the record and the
    oracle's solution as a global array."""
    import numpy as np

    import oracle as O
    import workloads as W

    boxes = cfg["boxes"]
    lev = O.make_level(boxes, W.domain_box(cfg["n"]), cfg["periodic"], 1.0, 1.0, None,
                       [W.scatter_faces(cfg["faces"][d], boxes, d) for d in range(3)])
    levels = O.build_levels(lev, 4, bool(args.aggregate))
    phi = O.new_cell_data(lev)
    opts = O.Opts(aggregate=bool(args.aggregate))
    log("oracle: whole solve at 256^3 on the host ...", q)
    c0 = os.times()
    t0 = time.perf_counter()
    info = O.solve(lev, phi, f_boxes, 1e-10, opts=opts, levels=levels)
    wall = time.perf_counter() - t0
    c1 = os.times()
    cpu_s = (c1.user - c0.user) + (c1.system - c0.system)
    log(f"oracle: {info['iters']} cycles in {wall:.1f} s ({cpu_s / wall:.2f} cores busy)", q)
    assert info["converged"]
    rec = {"value": wall * 1e3, "unit": "ms", "cores": max(1, int(round(cpu_s / wall))),
           "kind": "oracle",
           "sample": "one whole oracle.solve of this workload (256^3, 64 boxes, FP64 V-cycles "
                     "to max-norm 1e-10 from phi = 0), not scaled",
           "cycles": info["iters"], "final_rel_resid": info["history"][-1] / info["normf"],
           "cpu_seconds": cpu_s, "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}
    return rec, W.gather_cells(phi, boxes, cfg["n"], ng=1)


if __name__ == "__main__":
    main()
