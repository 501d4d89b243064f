#!/usr/bin/env python3
"""Benchmark of the Kronecker-sum Hubbard ground-state path on one MI355X.

Workload (default): periodic chain M=14, t=1, N_up=N_dn=7 (dim 3432^2 =
11,778,624), U in {2, 4, 8} -- the chain of the paper's Table IV.
One step = the whole hot path for the three U values, model parameters on the
host, everything else on the GPU:
  1. sector set-up: bases, H_up = H_dn in CSR and sliced ELL, site energies;
  2. plain FP64 Lanczos to E0 (Ritz residual <= 1e-12 |E0|);
  3. mixed Lanczos: FP32 vectors and products, FP64 alpha/beta, full
     reorthogonalisation with FP64 coefficients, FP64 tridiagonal solve,
     eigenvector from the stored basis, FP64 refinement (Rayleigh quotient);
  4. mixed Lanczos without reorthogonalisation (eigenvector by second pass,
     FP64 refinement).
Every product launch inside the timed steps is bracketed by HIP events on the
stream it runs on (the caller's current stream).  Time-to-E0 is the wall time
until the lowest Ritz value is within 1e-6 relative of the oracle's E0 (the
solves then continue to their stopping tests).  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# HIP events bracket every TIME_EVERY-th product launch of a solve (an event
# record between kernels delays the next one by a few microseconds)
TIME_EVERY = 8
TABLE4_M14_U4 = -8.0883491038  # Sec. V, Table IV (printed digits)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle sample time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 4x4-torus product timing")
    ap.add_argument("--copy-reference", type=int, default=0,
                    help="profiling aid: copy a buffer of this many MiB three times (counter calibration)")
    ap.add_argument("--lanczos-only", type=str, default="",
                    help="run one FP64 and one mixed solve of the named workload and exit (counter runs)")
    ap.add_argument("--matvec-only", type=str, default="",
                    help="profiling aid: 'workload:count' times count back-to-back products per dtype")
    return ap.parse_args()


def product_timing(hub, torch, model, reps=10):
    """Average event time of back-to-back products on the current stream."""
    sec = hub.Sector(model)
    out = {}
    for dt, name in ((hub.F32, "f32"), (hub.F64, "f64")):
        x = sec.start_vector(seed=1, dtype=dt)
        y = sec.empty(dt)
        sec.matvec(x, y)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            sec.matvec(x, y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        b = sec.matvec_bytes(dt)
        out[name] = {"avg_ms": ms, "bytes_per_launch": b, "GBps": b / ms / 1e6, "frac": b / ms / 1e6 / HBM_PEAK_GBPS}
        del x, y
    out["dim"] = sec.dim
    sec.close()
    return out


def ladder_mixed(hub, torch, model):
    """The 2x9 ladder (N = 9/9, dim 2.36e9): FP32 vectors and products with FP64
    scalars, plain recurrence, then the FP64 refinement of the eigenpair; the
    FP32 Ritz value against the FP64 Rayleigh quotient."""
    sec = hub.Sector(model)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = sec.ground_state(dtype=hub.F32, reorth=False, refine=True, tol=1e-7, max_iter=400)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    i = g.info
    out = {"dim": sec.dim, "iters": i["iters"], "solve_s": dt, "e0_ritz_fp32": i["e0_ritz"],
           "e0_refined_fp64": i["e0_refined"],
           "rel_err_ritz_vs_refined": abs(i["e0_ritz"] - i["e0_refined"]) / abs(i["e0_refined"]),
           "true_residual_fp64": i["true_residual"]}
    del g
    sec.close()
    return out


def square_mixed_gradients(hub, torch, model):
    """Config of the 4x4 torus (N = 7/7, dim 1.31e8, random t): FP32-mixed plain
    Lanczos with FP64 refinement, then the adjoint bilinear forms on psi, i.e.
    dE0/dt for the 32 bonds, dE0/dU_i and dE0/deps_i (Hellmann-Feynman). The
    Euler identity sum t dE/dt + sum U dE/dU + sum eps dE/deps = E (H is linear
    and homogeneous in its parameters) checks them."""
    import numpy as np
    sec = hub.Sector(model)
    # time-to-E0 against the FP64 GPU value (no oracle value exists at this size)
    e_ref = sec.ground_state(dtype=hub.F64, want_vector=False, tol=1e-10, max_iter=2000).e0
    g64 = sec.ground_state(dtype=hub.F64, want_vector=False, tol=1e-8, max_iter=2000, e0_target=e_ref,
                           e0_target_rel=1e-6)
    # the FP32 fused product's shape is tuned on its first use: keep that out of the timed solve
    sec.ground_state(dtype=hub.F32, want_vector=False, max_iter=2, allow_not_converged=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = sec.ground_state(dtype=hub.F32, reorth=False, refine=True, tol=1e-7, max_iter=600, e0_target=e_ref,
                         e0_target_rel=1e-6)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    db, dU, de = sec.param_bilinear(g.psi, g.psi)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    tvec = sec.bonds()[2]  # canonical bonds, in the order of db
    euler = float(np.dot(tvec, db) + np.dot(model.U, dU) + np.dot(model.eps, de))
    i = g.info
    out = {"dim": sec.dim, "iters": i["iters"], "solve_s": t1 - t0, "gradient_s": t2 - t1,
           "e0_ritz_fp32": i["e0_ritz"], "e0_refined_fp64": i["e0_refined"],
           "rel_err_ritz_vs_refined": abs(i["e0_ritz"] - i["e0_refined"]) / abs(i["e0_refined"]),
           "true_residual_fp64": i["true_residual"], "dE_dU_sum": float(np.sum(dU)),
           "e0_ref_fp64": e_ref,
           "time_to_e0_s": {"fp64_plain": g64.info["seconds_to_target"], "mixed_plain": i["seconds_to_target"]},
           "iters_to_e0": {"fp64_plain": g64.info["iters_to_target"], "mixed_plain": i["iters_to_target"]},
           "euler_identity_rel": abs(euler - i["e0_refined"]) / abs(i["e0_refined"])}
    del g
    sec.close()
    return out


def batch_timing(hub, torch, count=64):
    """The synthetic impurity-model batch (one DMFT step's exact-diagonalisation
    solves): one batched FP64 solve and one FP32 solve with FP64 refinement,
    against the same sectors solved one after another; plus one batched product."""
    import workloads as W
    models = W.aim_batch(count)
    secs = [hub.Sector(m) for m in models]
    batch = hub.Batch(secs)
    kw = dict(tol=1e-12, max_iter=400, check_every=5)
    batch.ground_state(dtype=hub.F64, **kw)  # tunes the product tiles
    batch.ground_state(dtype=hub.F32, tol=1e-7, refine=True, max_iter=400, check_every=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_b, it_b, _, info = batch.ground_state(dtype=hub.F64, **kw)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    e_m, _, _, _ = batch.ground_state(dtype=hub.F32, tol=1e-7, refine=True, max_iter=400, check_every=5)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    t0 = time.perf_counter()
    e_s = [s.ground_state(dtype=hub.F64, want_vector=False, **kw).e0 for s in secs]
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    x = batch.empty(hub.F64)
    x.fill_(1.0)
    y = batch.empty(hub.F64)
    batch.matvec(x, y)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        batch.matvec(x, y)
    ev1.record()
    torch.cuda.synchronize()
    mv_ms = ev0.elapsed_time(ev1) / 10
    mv_bytes = sum(s.matvec_bytes(hub.F64) for s in secs)
    out = {"sectors": count, "total_dim": batch.total, "max_dim": int(max(s.dim for s in secs)),
           "batch_fp64_s": t_b, "batch_f32_refined_s": t_m, "sequential_fp64_s": t_s,
           "batch_speedup_fp64": t_s / t_b, "steps": info["steps"], "graph_replays": info["graph_replays"],
           "max_iters": int(it_b.max()), "tile_columns": info["tile_columns"], "block_size": info["block_size"],
           "max_abs_diff_batch_vs_sequential": float(max(abs(a - b) for a, b in zip(e_b, e_s))),
           "max_abs_diff_refined_vs_fp64": float(max(abs(a - b) for a, b in zip(e_m, e_b))),
           "product_f64_ms": mv_ms, "product_f64_GBps": mv_bytes / mv_ms / 1e6}
    del x, y
    batch.close()
    for s in secs:
        s.close()
    return out


def greens_timing(hub, torch, model, steps=150):
    """Zero-temperature G_up(0, z) on the ring: ground state, then the particle
    and hole continued fractions (N+1 and N-1 sectors built inside the call)."""
    import numpy as np
    sec = hub.Sector(model)
    gs = sec.ground_state(dtype=hub.F64, tol=1e-13, want_vector=True, max_iter=600)
    z = 0.5 * float(model.U[0]) + 1j * np.pi * (2 * np.arange(32) + 1) / 10.0
    sec.greens_function(gs.e0, gs.psi, 0, 0, z[:1], max_steps=8)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, info, _ = sec.greens_function(gs.e0, gs.psi, 0, 0, z, max_steps=steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"site": 0, "spin": "up", "max_steps": steps, "seconds": dt, "steps_particle": info["steps_particle"],
           "steps_hole": info["steps_hole"], "sum_rule": info["norm2_particle"] + info["norm2_hole"],
           "max_abs_re_G_at_U/2+iw": float(np.max(np.abs(g.real)))}
    sec.close()
    return out


def k0_timing(hub, torch, model):
    """The same ring in its k = 0 translation block (Sec. VI): FP64 solve time and
    product time beside the full sector."""
    sec = hub.Sector(model, translation=1)
    g = sec.ground_state(dtype=hub.F64, tol=1e-12, want_vector=False, max_iter=600)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = sec.ground_state(dtype=hub.F64, tol=1e-12, want_vector=False, max_iter=600, time_kernels=TIME_EVERY)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"dim_k0": sec.dim, "e0_k0": g.e0, "iters": g.info["iters"], "solve_s": dt,
           "product_ms": g.info["matvec_ms"] / max(1, g.info["matvec_timed"])}
    sec.close()
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the product and the solver run on one GPU only; sharding V by column "
                                   "blocks over several GPUs is designed but not implemented",
                          "n_gpus": max(args.gpus, world)}))
        sys.exit(2)

    import torch

    import paper_1307_7542_amd as hub
    import workloads as W

    torch.cuda.set_device(0)
    F64, F32 = hub.F64, hub.F32

    if args.copy_reference:
        n = args.copy_reference * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copied {args.copy_reference} MiB x3", flush=True)
        return

    if args.lanczos_only:
        # the solver path alone (for counter runs of the fused product): one FP64 and one mixed solve
        name = args.lanczos_only
        sec = hub.Sector(W.config(name))
        for dt in (F64, F32):
            g = sec.ground_state(dtype=dt, want_vector=False, tol=1e-12 if dt == F64 else 1e-7)
            torch.cuda.synchronize()
            print(f"{name} lanczos dtype={'f64' if dt == F64 else 'f32'} iters={g.info['iters']}", flush=True)
        sec.close()
        return

    if args.matvec_only:
        name, cnt = args.matvec_only.split(":")
        sec = hub.Sector(W.config(name))
        for dt in (F32, F64):
            x = sec.start_vector(seed=1, dtype=dt)
            y = sec.empty(dt)
            for _ in range(int(cnt)):
                sec.matvec(x, y)
            torch.cuda.synchronize()
            print(f"{name} matvec dtype={'f32' if dt == F32 else 'f64'} launches={cnt}", flush=True)
        sec.close()
        return

    Us = (2, 4, 8)
    models = {U: W.config(f"ring14_u{U}") for U in Us}

    # E_ref for time-to-E0 (|theta - E_ref| <= 1e-6 |E_ref|): the stored oracle energies
    oracle_e0 = {}
    try:
        with open(os.path.join(ROOT, "tests", "golden", "oracle_values.json")) as f:
            ov = json.load(f)["entries"]
        oracle_e0 = {U: ov[f"ring14_u{U}"]["e0"] for U in Us}
    except (OSError, KeyError, ValueError):
        pass
    tgt = {U: dict(e0_target=oracle_e0.get(U), e0_target_rel=1e-6) for U in Us}

    def one_step():
        rec = {}
        for U, model in models.items():
            r = {}
            t0 = time.perf_counter()
            sec = hub.Sector(model)
            torch.cuda.synchronize()
            r["setup_s"] = time.perf_counter() - t0
            runs = {
                "fp64_plain": sec.ground_state(dtype=F64, want_vector=False, tol=1e-12, time_kernels=TIME_EVERY,
                                               **tgt[U]),
                "mixed_reorth": sec.ground_state(dtype=F32, reorth=True, refine=True, tol=1e-7,
                                                 time_kernels=TIME_EVERY, **tgt[U]),
                "mixed_plain": sec.ground_state(dtype=F32, reorth=False, refine=True, tol=1e-7,
                                                time_kernels=TIME_EVERY, **tgt[U]),
            }
            torch.cuda.synchronize()
            r["runs"] = {k: {"e0": v.e0, **v.info} for k, v in runs.items()}
            r["bytes"] = {"f64": sec.matvec_bytes(F64), "f32": sec.matvec_bytes(F32)}
            r["dim"] = sec.dim
            sec.close()
            rec[U] = r
        return rec

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    recs = [one_step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    # per dtype: event time, launches and algorithmic bytes of the launched product kernels
    # (when the first Lanczos update is fused into the product, its kernel also reads v_prev)
    agg = {"f64": [0.0, 0, 0, 0], "f32": [0.0, 0, 0, 0]}
    total_bytes = 0
    fused = {"f64": False, "f32": False}
    for rec in recs:
        for U, r in rec.items():
            for k, v in r["runs"].items():
                key = "f64" if k.startswith("fp64") else "f32"
                agg[key][0] += v["matvec_ms"]
                agg[key][1] += v["matvec_count"]
                agg[key][2] += v["matvec_count"] * v["matvec_bytes"]
                agg[key][3] += v["matvec_timed"]
                fused[key] = fused[key] or v["matvec_bytes"] > r["bytes"][key]
                total_bytes += v["matvec_count"] * r["bytes"][key]
    last = recs[-1]
    kern = {}
    for key in ("f64", "f32"):
        ms, cnt, kb, timed = agg[key]
        if cnt and timed:
            avg = ms / timed
            kern[key] = {"avg_ms": avg, "launches": cnt, "timed_launches": timed, "est_total_ms": avg * cnt,
                         "bytes_per_launch": kb / cnt, "GBps": (kb / cnt) / (avg * 1e-3) / 1e9,
                         "fused_lanczos_update": fused[key]}
    dom = max(kern, key=lambda k: kern[k]["est_total_ms"])

    per_U = {}
    for U in Us:
        r = last[U]
        e_ref = r["runs"]["fp64_plain"]["e0"]
        per_U[f"U={U}"] = {
            "e0_fp64": e_ref,
            "e0_oracle": oracle_e0.get(U),
            "rel_err_fp64_vs_oracle": (abs(e_ref - oracle_e0[U]) / abs(oracle_e0[U])) if U in oracle_e0 else None,
            "time_to_e0_s": {k: v["seconds_to_target"] for k, v in r["runs"].items()},
            "iters_to_e0": {k: v["iters_to_target"] for k, v in r["runs"].items()},
            "time_to_stop_test_s": {k: v["seconds_to_e0"] for k, v in r["runs"].items()},
            "solve_s": {k: v["seconds"] for k, v in r["runs"].items()},
            "iters": {k: v["iters"] for k, v in r["runs"].items()},
            "rel_err_vs_fp64": {k: abs(v["e0"] - e_ref) / abs(e_ref) for k, v in r["runs"].items()},
            "rel_err_ritz_vs_fp64": {k: abs(v["e0_ritz"] - e_ref) / abs(e_ref) for k, v in r["runs"].items()},
            "setup_s": r["setup_s"],
        }

    out = {
        "metric": "H·v GB/s & %HBM peak; Lanczos time-to-E0 mixed vs FP64 at |ΔE0|≤1e-6",
        "value": total_bytes / wall / 1e9,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "ring14 (periodic chain M=14, t=1, U in {2,4,8}, N_up=N_dn=7)",
                   "dim": last[Us[0]]["dim"], "start_seed": 7542, "vector_bytes_f32": last[Us[0]]["dim"] * 4,
                   "note": "vectors (47 MB FP32 / 94 MB FP64) fit in the 256 MB MALL"},
        "roofline": {"bound": "hbm", "achieved": kern[dom]["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": kern[dom]["GBps"] / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": (f"k_kron_quad<{'double' if dom == 'f64' else 'float'}> "
                                + ("fused with the first Lanczos update (reads v, v_prev; writes w)"
                                   if fused[dom] else "(reads v; writes H v)")),
                     "bytes_per_launch": kern[dom]["bytes_per_launch"], "avg_launch_ms": kern[dom]["avg_ms"]},
        "products": kern,
        "per_U": per_U,
        "time_to_e0": {
            "definition": "wall time from hub_ground_state entry until the lowest Ritz value is within 1e-6 "
                          "relative of the oracle E0 (checked every step, overlapped with the next step)",
            **{f"U={U}": {**per_U[f"U={U}"]["time_to_e0_s"],
                          "mixed_plain_over_fp64": (per_U[f"U={U}"]["time_to_e0_s"]["mixed_plain"] /
                                                    per_U[f"U={U}"]["time_to_e0_s"]["fp64_plain"])
                          if per_U[f"U={U}"]["time_to_e0_s"]["fp64_plain"] > 0 else None}
               for U in Us},
        },
        "table4_check": {"U": 4, "printed_E_min": TABLE4_M14_U4,
                         "e0_fp64": last[4]["runs"]["fp64_plain"]["e0"]},
        "paper_context": {"note": "one intel i7 (model, cores, precision unstated); not like-for-like",
                          "table4_ring14_lanczos_s": {"two_spin_binary_search": 3459.85,
                                                      "one_spin_binary_search": 702.15,
                                                      "one_spin_stored_index": 701.42},
                          "table2_ring14_offdiag_generation_s": {"two_spin": 5.02, "one_spin": 0.55},
                          "generation_speedup_claim": "1/9 to 1/11"},
    }
    # HBM traffic of the dominant product from the committed counter run, only
    # while the product source is unchanged since the counters were taken
    try:
        import hashlib
        with open(os.path.join(ROOT, "profiles", "k_kron_fused_counters.json")) as f:
            cj = json.load(f)
        with open(os.path.join(ROOT, "paper_1307_7542_amd", "csrc", "matvec.hip"), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        ent = cj["kernels"].get(f"ring14_u4:{dom}" + (":fused" if fused[dom] else ""))
        if ent and cj.get("matvec_source_sha256") == sha:
            out["roofline"]["traffic"] = ent["traffic_bytes"]
            out["roofline"]["traffic_note"] = ("FETCH_SIZE x %.3f + WRITE_SIZE x %.3f per launch (copy-kernel "
                                               "calibration), U=4, counters taken on %s; %s"
                                               % (cj["calibration"]["fetch_scale"], cj["calibration"]["write_scale"],
                                                  ent["kernel"], cj.get("shape_note", "")))
    except (OSError, KeyError, ValueError):
        pass
    if not args.no_extra:
        out["products_square4x4"] = product_timing(hub, torch, W.config("square4x4"))
        out["lanczos_square4x4_mixed_gradients"] = square_mixed_gradients(hub, torch, W.config("square4x4"))
        out["products_ladder2x9"] = product_timing(hub, torch, W.config("ladder2x9"), reps=3)
        out["lanczos_ladder2x9_mixed"] = ladder_mixed(hub, torch, W.config("ladder2x9"))
        out["aim_batch64"] = batch_timing(hub, torch)
        out["greens_ring14_u4"] = greens_timing(hub, torch, models[4])
        out["k0_ring14_u4"] = k0_timing(hub, torch, models[4])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(models[4], args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline(model, target_s):
    """The oracle as it stands (two-spin basis, binary-search indexing, FP64),
    timed on a bounded sample of the same workload: whole products (all rows,
    matrix-free) repeated until about target_s seconds of CPU work."""
    import numpy as np

    import oracle
    osec = oracle.Sector(model, explicit_keys=False)
    rows = np.arange(osec.dim, dtype=np.int64)
    x = oracle.start_vector(7542, osec.dim)
    t = time.perf_counter()
    osec.apply_rows(rows, x)
    one = time.perf_counter() - t
    reps = max(1, int(round(target_s / max(one, 1e-9))) - 1)
    t = time.perf_counter()
    for _ in range(reps):
        osec.apply_rows(rows, x)
    dt = time.perf_counter() - t
    rate = reps * osec.dim / dt
    return {"value": rate * 16 / 1e9, "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{reps} whole FP64 products of ring14 U=4 ({osec.dim} rows each; two-spin matrix-free rows "
                      f"with binary-search indexing) after one warm-up product, {dt:.1f} s; GB/s = rows/s x 16 B "
                      f"(8 B read + 8 B written per element)",
            "rows_per_s": rate, "product_s": dt / reps}


if __name__ == "__main__":
    main()
