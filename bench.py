"""Benchmark: factor time and RHS/s of the butterfly-compressed multifrontal
solver on one MI355X, with the roofline of the dominant kernel and the CPU
oracle timed on a bounded sample of the same workload.

One step = bfmf_factor (all fronts) + bfmf_solve of the workload's RHS block
(GMRES to a true relative residual <= 1e-3), inputs resident in HBM.
value = RHS per second of whole steps (factorization included).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"fp64_tflops": 78.6, "fp32_tflops": 157.3, "hbm_gbs": 8000.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="helmholtz100")
    ap.add_argument("--n", type=int, default=None, help="override the grid size")
    ap.add_argument("--form", default="batched", choices=["batched", "plain"])
    ap.add_argument("--precision", default=None, choices=["c128", "c64"], help="default: the workload's")
    ap.add_argument("--n-min", type=int, default=None, help="compression threshold (0: exact)")
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--cpu-baseline-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form comparison step")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--serve-seconds", type=float, default=0.25, help="arrival window of the serving run")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="mean request arrivals per second")
    ap.add_argument("--sep-leaf", type=int, default=None,
                    help="separators are bisected down to this many nodes (HOD-BF leaves); default: the workload's")
    ap.add_argument("--parallel-levels", type=int, default=0,
                    help="separator variant: the top levels of the dissection cut across one axis (parallel planes)")
    ap.add_argument("--direct", action="store_true",
                    help="direct mode: X = M^-1 B from the factorization, no GMRES (use with a tight --tol)")
    ap.add_argument("--gemm-tile", type=int, default=-1,
                    help="force one grouped-GEMM tile shape (0..5; -1: the autotuned choice per launch)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="profiling: measure the tile tables on a small problem, then run two streaming kernels "
                         "of known size (an elementwise negation and a device copy, each reading and writing this "
                         "many MiB) that scale HBM byte counters and mark where the workload's dispatches begin")
    return ap.parse_args()


def prime_tile_tables(bfmf):
    """A small compressed factorization in both precisions: the grouped-GEMM tile tables of this
    device are measured here, so that a profile taken after it sees only the workload's launches."""
    from workloads import helmholtz_7pt
    rp, ci, v, _ = helmholtz_7pt((12, 12, 12), 0.05)
    for prec in (bfmf.BFMF_C128, bfmf.BFMF_C64_MIXED):
        s = bfmf.Solver(0).analyze(rp, ci, v, dims=(12, 12, 12), leaf_max=64, sep_leaf=16)
        s.factor(tol=1e-3, n_min=40, batched=True, precision=prec)
        s.close()


def calibrate_copy(mib):
    """Streaming kernels of known traffic: dst = -src (an elementwise kernel) and dst = src (a
    device-to-device copy), each reading mib MiB and writing mib MiB."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()
    print(f"[bench] calibration kernels: {mib} MiB read + {mib} MiB written each", file=sys.stderr, flush=True)


def cpu_baseline(prob, budget_s, nrhs, parallel_levels=0):
    """Oracle (NumPy/SciPy FP64) factorization of the same workload, stopped
    after about budget_s seconds of fronts in postorder; scaled to the whole
    factorization by algorithmic flops, plus the sampled solve cost."""
    from oracle import nd, multifrontal as mf
    from oracle.symbolic import symbolic
    od = nd.nd_grid(prob.dims, leaf_max=512, sep_leaf=64, parallel_levels=parallel_levels)
    sym = symbolic(prob.rowptr, prob.colind, od)
    total = sum(mf.front_flops(od, sym, f) for f in range(od.nfronts))
    t0 = time.perf_counter()
    fac = mf.factor(prob.rowptr, prob.colind, prob.values, od, sym, stop_seconds=budget_s)
    t_f = time.perf_counter() - t0
    done = sum(mf.front_flops(od, sym, f) for f in range(fac.done))
    est_factor = t_f * total / max(done, 1.0)
    # the solve touches every factor entry once per RHS: scale by factor storage
    sizes = [(float(od.send[f] - od.sbeg[f]), float(sym.Iu[f].shape[0])) for f in range(od.nfronts)]
    store = sum(ns * ns + 2 * ns * nu for ns, nu in sizes)
    store_done = sum(ns * ns + 2 * ns * nu for ns, nu in sizes[:fac.done])
    t0 = time.perf_counter()
    Bs = prob.rhs[:, :1]
    _ = _partial_solve(fac, Bs, fac.done)
    t_s = (time.perf_counter() - t0) * store / max(store_done, 1.0) * nrhs
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    value = nrhs / (est_factor + t_s)
    return {"value": value, "unit": "RHS/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle multifrontal LU of the first {fac.done} of {od.nfronts} fronts (postorder) of the "
                      f"same grid in {t_f:.1f} s ({100 * done / total:.2f}% of the flops), and their sweeps for "
                      f"1 RHS; scaled to the whole factorization by flops and to {nrhs} RHS by factor storage",
            "est_factor_s": est_factor, "est_solve_s": t_s}


def _partial_solve(fac, B, nfr):
    import scipy.linalg as sla
    from oracle import multifrontal as mf
    od, sym = fac.od, fac.sym
    y = B[od.perm, :].copy()
    for f in range(nfr):
        b, e = int(od.sbeg[f]), int(od.send[f])
        z = y[b:e, :][mf.swaps_to_perm(fac.piv[f]), :]
        z = sla.solve_triangular(fac.lu[f], z, lower=True, unit_diagonal=True)
        y[b:e, :] = z
        if sym.Iu[f].shape[0]:
            y[sym.Iu[f], :] -= fac.F21[f] @ z
    return y


def run_form(bfmf, s, prob, nrhs, dB, dX, steps, warmup, form, precision, n_min, tol, timing=True, direct=False):
    """Factor + GMRES solve of the RHS block (or, direct, one application of the factorization),
    `steps` timed steps after `warmup` untimed ones."""
    import torch
    prec = bfmf.BFMF_C128 if precision == "c128" else bfmf.BFMF_C64_MIXED
    so = bfmf.bfmf_default_solve_opts()
    so.true_rtol = 1e-3
    if direct:
        so.max_iter = -1

    def step():
        s.factor(tol=tol, n_min=n_min, precision=prec, batched=(form == "batched"), timing=timing)
        o, st = bfmf.bfmf_solve_device(s.h, dB.data_ptr(), prob.n, dX.data_ptr(), prob.n, nrhs, so)
        if st != 0:
            raise RuntimeError(f"solve did not converge ({form}, {precision}): relres {o.relres_max}")
        return o

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    bfmf.bfmf_reset_kernel_stats(s.h)
    t0 = time.perf_counter()
    fsec, ssec, iters, relres = [], [], [], []
    for _ in range(steps):
        o = step()
        fsec.append(s.stats()["factor_seconds"])
        ssec.append(o.seconds)
        iters.append(o.iters_max)
        relres.append(o.relres_max)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    st = s.stats()
    return {"T": T, "value": nrhs * steps / T, "ms_per_step": 1e3 * T / steps,
            "factor_s": float(np.mean(fsec)), "solve_s": float(np.mean(ssec)),
            "solve_rhs_per_s": nrhs / float(np.mean(ssec)), "gmres_iters": int(max(iters)),
            "relres_max": float(max(relres)), "factor_flops": st["factor_flops"],
            "factor_bytes": st["factor_bytes"], "dense_factor_bytes": st["dense_factor_bytes"],
            "max_rank": st["max_rank"], "kernels": s.kernel_stats(), "gemm_tiles": s.gemm_tile_launches()}


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "kernels_helmholtz100_c64.md")


def library_sources_sha256():
    """Hash of every library source (kernels, launch plans, tile tables): traffic counted by the
    profiler describes these sources only."""
    import hashlib
    base = os.path.join(ROOT, "paper_2007_00202_amd", "csrc")
    h = hashlib.sha256()
    for dirpath, _, files in sorted(os.walk(base)):
        for f in sorted(files):
            if f.endswith((".hip", ".hpp", ".cpp", ".h")):
                path = os.path.join(dirpath, f)
                h.update(os.path.relpath(path, base).encode())
                h.update(open(path, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, precision):
    """HBM bytes per launch of `kernel` from the committed profiler record (FETCH_SIZE and
    WRITE_SIZE scaled by a copy of known size), or None when the record is missing, is for
    another kernel or precision, or the library sources changed since it was taken."""
    if precision != "c64" or not os.path.exists(TRAFFIC_RECORD):
        return None
    for line in open(TRAFFIC_RECORD):
        if line.startswith("* record: "):
            rec = json.loads(line[len("* record: "):])
            if rec.get("kernel") == kernel and rec.get("sources_sha256") == library_sources_sha256():
                return rec.get("traffic_bytes_per_launch")
    return None


def roofline(ks, steps, precision):
    """Roofline of the dominant single-kernel class (estimated total time; sampled classes scaled)."""
    single = {"assemble": "hbm", "schur_gemm": "mfma", "butterfly_gemm": "mfma", "interp_decomp": "alu",
              "entry_extract": "hbm"}

    def total_s(k):
        v = ks[k]
        return v["seconds"] * v["launches_all"] / max(v["launches"], 1)

    dom = max(single, key=total_s)
    kk = ks[dom]
    per_launch_s = kk["seconds"] / max(kk["launches"], 1)
    bound = single[dom]
    fp_peak = PEAKS["fp64_tflops"] if precision == "c128" else PEAKS["fp32_tflops"]
    if bound == "hbm":
        ach = kk["bytes"] / max(kk["seconds"], 1e-30) / 1e9
        peak, unit = PEAKS["hbm_gbs"], "GB/s"
    else:  # MFMA contraction, or FP64 vector arithmetic (the ID kernel) against the FP64 peak
        ach = kk["flops"] / max(kk["seconds"], 1e-30) / 1e12
        peak, unit = (fp_peak if bound == "mfma" else PEAKS["fp64_tflops"]), "TFLOP/s"
    rf = {"bound": bound, "kernel": dom, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
          "traffic": measured_traffic(dom, precision), "timed_launches": kk["launches"],
          "launches": kk["launches_all"],
          "avg_launch_ms": 1e3 * per_launch_s}
    kernels = {k: {"ms": 1e3 * total_s(k) / steps, "launches": v["launches_all"] // max(steps, 1),
                   "timed_launches": v["launches"] // max(steps, 1),
                   "tflops": v["flops"] / max(v["seconds"], 1e-30) / 1e12,
                   "gbs": v["bytes"] / max(v["seconds"], 1e-30) / 1e9}
               for k, v in ks.items() if v["launches_all"]}
    return rf, kernels


def run_serving(bfmf, seconds, rate, max_rhs, precision):
    """Three resident factorizations (48^3, 64^3, 80^3) answer a seeded Poisson
    stream of point-source requests; latency from submission to solution."""
    import threading
    from workloads import make_problem, request_stream, rng_for
    from workloads.configs import serving_grids
    prec = bfmf.BFMF_C128 if precision == "c128" else bfmf.BFMF_C64_MIXED
    solvers, sizes = [], []
    for g in serving_grids():
        p = make_problem("helmholtz100", n=g, nrhs=1, config_id="serving")
        sv = bfmf.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims)
        sv.factor(tol=1e-3, n_min=1024, precision=prec, batched=True)
        solvers.append(sv)
        sizes.append(p.n)
    srv = bfmf.Server(0, max_batch_rhs=max_rhs, result_bytes=24 << 30, true_rtol=1e-3)
    ids = [srv.attach(sv) for sv in solvers]
    stream = request_stream(rate, seconds, sizes, max_rhs, rng_for("serving", "arrivals"))
    tickets = [None] * len(stream)
    base = srv.clock()

    def producer():
        for k, (t, m, rows) in enumerate(stream):
            dt = base + t - srv.clock()
            if dt > 0:
                time.sleep(dt)
            tickets[k] = srv.submit_points(ids[m], rows)

    th = threading.Thread(target=producer)
    th.start()
    infos = []
    for k in range(len(stream)):
        while tickets[k] is None:
            time.sleep(0.0005)
        infos.append(srv.wait(tickets[k]))
    th.join()
    srv.close()
    for sv in solvers:
        sv.close()
    bad = [i for i in infos if i["status"] != 0]
    lat = np.array([i["t_done"] - i["t_submit"] for i in infos])
    first = min(i["t_submit"] for i in infos)
    last = max(i["t_done"] for i in infos)
    nrhs = sum(i["nrhs"] for i in infos)
    return {"grids": [f"{g}^3" for g in serving_grids()], "precision": precision, "offered_req_per_s": rate,
            "window_s": seconds, "requests": len(infos), "rhs": int(nrhs), "failed": len(bad),
            "rhs_per_s": nrhs / (last - first), "makespan_s": last - first,
            "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "mean_batch_rhs": float(np.mean([i["batch_rhs"] for i in infos])),
            "max_iters": int(max(i["iters"] for i in infos)), "max_relres": float(max(i["relres"] for i in infos))}


def operator_label(cfg):
    if cfg.get("op") == "acoustic27":
        return "3D visco-acoustic 27-pt with absorbing layers"
    if cfg.get("omega") == 0.0:
        return "3D Poisson 7-pt"
    return "3D Helmholtz 7-pt"


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (sharding across GPUs is not implemented); --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2007_00202_amd import bfmf
    from workloads import make_problem, CONFIGS

    if a.calibrate_copy_mib > 0:  # profiling: tile tables first, then the calibration kernels as a marker
        prime_tile_tables(bfmf)
        calibrate_copy(a.calibrate_copy_mib)
    if a.gemm_tile >= 0:
        bfmf.bfmf_set_gemm_tile(a.gemm_tile)

    cfg = CONFIGS[a.config]
    if cfg["kind"] != "grid":
        print(json.dumps({"error": f"{a.config}: the benchmark runs the grid workloads"}))
        sys.exit(2)
    prob = make_problem(a.config, n=a.n)
    n_min = cfg["n_min"] if a.n_min is None else a.n_min
    tol = cfg["tol"] if a.tol is None else a.tol
    precision = a.precision or cfg["precision"]
    nrhs = prob.rhs.shape[1]
    sep_leaf = a.sep_leaf or cfg.get("sep_leaf", 64)
    s = bfmf.Solver(0).analyze(prob.rowptr, prob.colind, prob.values, dims=prob.dims, sep_leaf=sep_leaf,
                               parallel_levels=a.parallel_levels)
    dB = torch.from_numpy(np.ascontiguousarray(prob.rhs.T)).to("cuda")  # column-major (N, nrhs)
    dX = torch.zeros_like(dB)
    r = run_form(bfmf, s, prob, nrhs, dB, dX, a.steps, a.warmup, a.form, precision, n_min, tol, direct=a.direct)
    rf, kernels = roofline(r["kernels"], a.steps, precision)
    out = {
        "metric": "factor time + RHS/s at rel-residual <=1e-3",
        "value": r["value"],
        "unit": "RHS/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128" if precision == "c128" else "c64+f64",
        "data": "synthetic",
        "config": {"workload": f"{a.config}: {operator_label(cfg)} {prob.dims[0]}^3 (N={prob.n}), {nrhs} RHS",
                   "form": a.form, "n_min": n_min, "tol": tol, "precision": precision, "sep_leaf": sep_leaf,
                   "parallel_levels": a.parallel_levels,
                   "solver": "direct" if a.direct else "gmres"},
        "factor_s": r["factor_s"], "solve_s": r["solve_s"], "solve_rhs_per_s": r["solve_rhs_per_s"],
        "gmres_iters": r["gmres_iters"], "relres_max": r["relres_max"],
        "factor_tflops": r["factor_flops"] / r["factor_s"] / 1e12,
        "factor_gb": r["factor_bytes"] / 1e9, "dense_factor_gb": r["dense_factor_bytes"] / 1e9,
        "max_rank": r["max_rank"],
        "roofline": rf,
        "kernels": kernels,
        "gemm_tile_launches": {k: v // max(a.steps, 1) for k, v in r["gemm_tiles"].items()},
    }
    if not a.no_plain:  # the plain GPU form: complex128, fronts and constructions one at a time
        p = run_form(bfmf, s, prob, nrhs, dB, dX, 1, 0, "plain", "c128", n_min, tol, timing=False)
        out["plain"] = {"form": "plain", "precision": "c128", "value": p["value"], "factor_s": p["factor_s"],
                        "solve_s": p["solve_s"], "gmres_iters": p["gmres_iters"], "relres_max": p["relres_max"]}
    s.close()
    if not a.no_serve:
        out["serving"] = run_serving(bfmf, a.serve_seconds, a.serve_rate, 64, precision)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, a.cpu_baseline_seconds, nrhs, a.parallel_levels)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
