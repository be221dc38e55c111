"""Benchmark: time to 1e-8 relative error of RGDBEK on one MI355X.

Workload (default): dense inconsistent least squares, A 20000 x 5000 with
i.i.d. N(0,1) entries, b = A x* + r with r in null(A^T), ||r|| = 0.1 ||A x*||
(synthetic, seed 0).  One "step" is one full solve from x_0 = 0 to
||x - x*|| / ||x*|| <= 1e-8, inputs resident in HBM.  Two forms are timed:
plain FP64 and the mixed form (FP32 inner iterations, FP64 refinement); the
headline value is the faster one.  Also reported: the roofline of the
dominant kernel (the fused A x / A^T z pass, HBM-bound) timed with HIP events
on the stream it runs on, and the FP64 oracle timed on the host cores on a
bounded sample.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "time to 1e-8 rel. error + SpMV HBM GB/s; mixed/batched vs plain FP64 GPU"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=20000)
    ap.add_argument("--n", type=int, default=5000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--kc", type=int, default=0)
    ap.add_argument("--kr", type=int, default=0)
    ap.add_argument("--inner-tol", type=float, default=0.0)
    ap.add_argument("--inner-max", type=int, default=0)
    ap.add_argument("--tune", action="store_true",
                    help="sweep block sizes before timing (slow)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp64,mixed_f32")
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sparse pass and batched-form measurements")
    ap.add_argument("--probe-sparse", action="store_true",
                    help="counter-run program: copy calibration, then the "
                    "sparse residual passes on the power-law matrix")
    ap.add_argument("--probe", action="store_true",
                    help="counter probe: a 1 GiB device copy (calibration) "
                         "and fused-pass launches only, no solves")
    return ap.parse_args()


def probe(args):
    """Short program for hardware-counter runs: torch's device copy of a
    known size (FETCH_SIZE/WRITE_SIZE calibration), then the fused residual
    pass in FP64 and FP32 (rgdbek_apply) on the benchmark matrix."""
    import torch
    import paper_2509_19267_amd as rg
    dev = torch.device("cuda", 0)
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy: 1 GiB read + 1 GiB write per launch")
    from paper_2509_19267_amd import tune
    rng = np.random.default_rng(0)
    m, n = args.m, args.n
    a = torch.as_tensor(rng.standard_normal((m, n))).to(dev)
    for form, prec, dt in [("fp64", "f64", torch.float64),
                           ("mixed_f32", "f32", torch.float32)]:
        ch = tune.lookup("dense", m, n, form) or {}
        s = rg.Solver(a, k_col=8, k_row=8, precision="mixed_f32",
                      tile_rows=ch.get("tile_rows", 0))
        xv = torch.randn(n, dtype=dt, device=dev)
        zv = torch.randn(m, dtype=dt, device=dev)
        for _ in range(3):
            s.apply(xv, zv, precision=prec)
        torch.cuda.synchronize()
        log(f"fused pass {prec} (tile_rows {ch.get('tile_rows', 0)}): 3 launches")
        s.close()
    print(json.dumps({"probe": "done", "m": m, "n": n}))


def probe_sparse():
    """Short program for hardware-counter runs of the sparse path: the 1 GiB
    device copy (calibration), then three CSR + CSC residual pass pairs
    (rgdbek_apply) per precision on the 1,000,000 x 500,000 power-law
    matrix."""
    import torch
    import paper_2509_19267_amd as rg
    import workloads
    dev = torch.device("cuda", 0)
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    log("copy: 1 GiB read + 1 GiB write per launch")
    p = workloads.sparse_powerlaw(1_000_000, 500_000, mean_len=10,
                                  max_len=2000, seed=0)
    m, n = p.a.shape
    rp, ci, v = workloads.to_csr_arrays(p.a)
    csr = (torch.as_tensor(rp).to(dev), torch.as_tensor(ci).to(dev),
           torch.as_tensor(v).to(dev))
    s = rg.Solver(csr=csr, shape=(m, n), eta=0.1, precision="mixed_f32")
    for prec, dt in [("f64", torch.float64), ("f32", torch.float32)]:
        x = torch.randn(n, dtype=dt, device=dev)
        z = torch.randn(m, dtype=dt, device=dev)
        ax = torch.empty(m, dtype=dt, device=dev)
        atz = torch.empty(n, dtype=dt, device=dev)
        for _ in range(3):
            s.apply(x, z, ax, atz, precision=prec)
        torch.cuda.synchronize()
        log(f"sparse pass pair {prec}: 3 launches")
    s.close()
    print(json.dumps({"probe": "done", "m": m, "n": n, "nnz": int(p.a.nnz)}))


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dense_fused_pass_20000x5000_hbm.md")


def counted_traffic(prec, tile_rows, m, n):
    """HBM bytes per launch of the fused pass from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary (copy-calibrated); None when the summary is
    for another shape or row tile."""
    if (m, n) != (20000, 5000):
        return None
    try:
        with open(TRAFFIC_FILE) as f:
            line = [l for l in f if l.startswith("traffic_bytes_per_launch:")][0]
    except (OSError, IndexError):
        return None
    tb, tr = line.split("tile_rows:")
    vals = dict(kv.split("=") for kv in tb.split(":")[1].split())
    tiles = dict(kv.split("=") for kv in tr.split())
    if int(tiles.get(prec, -1)) != int(tile_rows or 0):
        return None
    return int(vals[prec])


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2509_19267_amd as rg
    from paper_2509_19267_amd import tune
    import workloads

    assert torch.cuda.is_available(), "bench needs a HIP device"
    if args.probe:
        probe(args)
        return
    if args.probe_sparse:
        probe_sparse()
        return
    dev = torch.device("cuda", 0)
    t0 = time.time()
    prob = workloads.dense_least_squares(args.m, args.n, seed=0)
    log(f"generated {args.m}x{args.n} least-squares problem in {time.time()-t0:.1f}s")
    a = torch.as_tensor(prob.a).to(dev)
    b = torch.as_tensor(prob.b).to(dev)
    xs = torch.as_tensor(prob.x_star).to(dev)
    stream = torch.cuda.Stream()

    form_list = args.forms.split(",")
    choices = {}
    for form in form_list:
        ch = tune.lookup("dense", args.m, args.n, form)
        if args.kc and args.kr:
            ch = dict(k_col=args.kc, k_row=args.kr, gram_aat=args.kr > 256,
                      inner_tol=args.inner_tol, inner_max=args.inner_max)
        if args.tune or ch is None:
            ch = tune.tune_dense(a, b, xs, stream=stream, log=log,
                                 precision=form)
        choices[form] = ch
        log(f"{form}: block sizes {ch}")

    forms = {}
    handles = {}
    for form in form_list:
        choice = choices[form]
        kw = dict(k_col=choice["k_col"], k_row=choice["k_row"],
                  gram_aat=choice.get("gram_aat", False), stop="err_ref",
                  tol=args.tol, max_iter=20000, precision=form, stream=stream,
                  inner_tol=choice.get("inner_tol", 0.0),
                  inner_max=choice.get("inner_max", 0),
                  tile_rows=choice.get("tile_rows", 0))
        tc = time.time()
        s = rg.Solver(a, **kw)
        create_s = time.time() - tc
        handles[form] = s
        for _ in range(args.warmup):
            s.solve(b, x_ref=xs)
        torch.cuda.synchronize()
        times, its, errs, evs = [], [], [], []
        torch.cuda.synchronize()
        for _ in range(args.steps):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            t1 = time.perf_counter()
            x, info = s.solve(b, x_ref=xs)
            times.append(time.perf_counter() - t1)
            ev1.record(stream)
            torch.cuda.synchronize()
            evs.append(ev0.elapsed_time(ev1))
            its.append(info["iterations"])
            errs.append(float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs)))
        ev_ms = float(np.mean(evs))
        forms[form] = dict(ms_per_solve=1e3 * float(np.mean(times)),
                           ms_min=1e3 * float(np.min(times)),
                           ms_events=ev_ms, iterations=int(np.median(its)),
                           outer=int(info["outer_iterations"]),
                           rel_err=float(np.max(errs)),
                           converged=bool(info["converged"]),
                           create_s=create_s, choice=choice)
        log(f"{form}: {forms[form]}")

    # roofline of the dominant kernel: the fused pass A x, A^T z (FP64 and,
    # for the mixed form, FP32), timed with events on the handle's stream
    m, n = args.m, args.n
    roof = {}
    for form, prec, vb in [("fp64", "f64", 8), ("mixed_f32", "f32", 4)]:
        if form not in handles:
            continue
        s = handles[form]
        dt = torch.float64 if prec == "f64" else torch.float32
        xv = torch.randn(n, dtype=dt, device=dev)
        zv = torch.randn(m, dtype=dt, device=dev)
        ax = torch.empty(m, dtype=dt, device=dev)
        atz = torch.empty(n, dtype=dt, device=dev)
        for _ in range(3):
            s.apply(xv, zv, ax, atz, precision=prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.apply_reps):
            s.apply(xv, zv, ax, atz, precision=prec)
        e1.record(stream)
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / args.apply_reps
        alg_bytes = m * n * vb + 2 * (m + n) * vb
        gbs = alg_bytes / (us * 1e-6) / 1e9
        roof[prec] = dict(us=us, alg_bytes=alg_bytes, gbs=gbs)
        log(f"fused pass {prec}: {us:.1f} us per launch, {gbs:.0f} GB/s")

    best_form = min(forms, key=lambda f: forms[f]["ms_per_solve"])
    best = forms[best_form]
    dom = "f32" if best_form == "mixed_f32" and "f32" in roof else "f64"
    r = roof.get(dom)
    roofline = None
    if r:
        dom_form = "mixed_f32" if dom == "f32" else "fp64"
        traffic = counted_traffic(dom, choices.get(dom_form, {}).get("tile_rows", 0),
                                  m, n)
        roofline = {"bound": "hbm", "achieved": round(r["gbs"], 1),
                    "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(r["gbs"] / PEAK_HBM_GBS, 4),
                    "traffic": traffic,
                    "kernel": f"dense_fused_kernel<{'float' if dom == 'f32' else 'double'}> (+finalize)",
                    "alg_bytes_per_launch": r["alg_bytes"],
                    "us_per_launch": round(r["us"], 2)}

    extras = None
    if not args.no_extras:
        for s in handles.values():
            s.close()
        handles = {}
        del a, b, xs
        torch.cuda.empty_cache()
        extras = {"spmv": spmv_powerlaw(), "batched": batched_laplacian(),
                  "gdbek_vs_rgdbek": gdbek_vs_rgdbek(), "fem": fem_table8(),
                  "differentiable": differentiable_dense(args.m, args.n)}

    cpu = None
    if not args.no_cpu_baseline:
        ref_form = "fp64" if "fp64" in forms else best_form
        cpu = cpu_baseline(prob, choices[ref_form], forms[ref_form]["iterations"])

    out = {
        "metric": METRIC, "value": round(best["ms_per_solve"], 3), "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(best["ms_per_solve"], 3),
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32+f64" if best_form == "mixed_f32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"dense_least_squares_{m}x{n}", "m": m, "n": n,
                   "tol": args.tol, "form": best_form,
                   **{k: v for k, v in choices[best_form].items()}},
        "forms": forms,
        "speedup_mixed_vs_fp64": (round(forms["fp64"]["ms_per_solve"] /
                                        forms["mixed_f32"]["ms_per_solve"], 3)
                                  if "fp64" in forms and "mixed_f32" in forms else None),
        "roofline": roofline,
        "roofline_all": roof,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out))
    for s in handles.values():
        s.close()


def spmv_powerlaw(reps=20):
    """Residual passes of the sparse path (CSR row pass + CSC column pass,
    rgdbek_apply) on the 1,000,000 x 500,000 power-law matrix, FP64 and FP32,
    timed with HIP events on the handle's stream; then 20 FP64 iterations of
    a solve on the same matrix (time per iteration of the whole path)."""
    import torch
    import paper_2509_19267_amd as rg
    import workloads
    p = workloads.sparse_powerlaw(1_000_000, 500_000, mean_len=10,
                                  max_len=2000, seed=0)
    m, n = p.a.shape
    nnz = p.a.nnz
    rp, ci, v = workloads.to_csr_arrays(p.a)
    st = torch.cuda.Stream()
    csr = (torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda(),
           torch.as_tensor(v).cuda())
    s = rg.Solver(csr=csr, shape=(m, n), eta=0.1, precision="mixed_f32",
                  stream=st)
    out = {"workload": f"sparse_powerlaw_{m}x{n}", "nnz": int(nnz)}
    for prec, dt, vb in [("f64", torch.float64, 8), ("f32", torch.float32, 4)]:
        x = torch.randn(n, dtype=dt, device="cuda")
        z = torch.randn(m, dtype=dt, device="cuda")
        ax = torch.empty(m, dtype=dt, device="cuda")
        atz = torch.empty(n, dtype=dt, device="cuda")
        torch.cuda.synchronize()
        for _ in range(3):
            s.apply(x, z, ax, atz, precision=prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            s.apply(x, z, ax, atz, precision=prec)
        e1.record(st)
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        # CSR pass: values + indices + row pointers + x + output; CSC pass
        # likewise with the roles of m and n swapped
        alg = 2 * nnz * (vb + 4) + 8 * (m + 1) + 8 * (n + 1) + 2 * vb * (m + n)
        out[prec] = {"us_per_pair": round(us, 1), "alg_bytes": int(alg),
                     "GB/s": round(alg / us / 1e3, 1),
                     "frac": round(alg / us / 1e3 / PEAK_HBM_GBS, 4)}
        log(f"sparse passes {prec}: {us:.1f} us per CSR+CSC pair, "
            f"{alg / us / 1e3:.0f} GB/s")
    s.close()
    # a short FP64 solve on the same matrix (eta = 0.1: blocks of 50 000
    # columns and 100 000 rows), block projections to 0.1 in at most 16
    # CG steps: the time per iteration of the whole sparse path
    b = torch.as_tensor(p.b).cuda()
    xs = torch.as_tensor(p.x_star).cuda()
    s = rg.Solver(csr=csr, shape=(m, n), eta=0.1, stop="err_ref", tol=1e-8,
                  max_iter=20, inner_tol=0.1, inner_max=16, stream=st)
    s.solve(b, x_ref=xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = s.solve(b, x_ref=xs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.close()
    out["solve_fp64"] = {"iterations": info["iterations"],
                         "ms_per_iteration": round(1e3 * el / max(info["iterations"], 1), 2),
                         "rel_err_after": info["final_metric"]}
    log(f"sparse solve: {out['solve_fp64']}")
    del csr
    torch.cuda.empty_cache()
    return out


def batched_laplacian(count=16, itol=0.1, imax=16, tol=1e-8):
    """Batched form vs the plain FP64 path on the same inputs: `count`
    shifted 2-D Laplacians with 20% extra rows (n from 2000 to 20000,
    values rounded to FP32 storage, planted x*), time to ||x - x*|| <= tol
    ||x*|| for every system: one batched FP64 solve, one batched mixed solve
    (FP32 values, FP64 refinement), and the systems one by one with the
    single-system FP64 solver.  Inner projections: tolerance itol, at most
    imax CG steps (the same for all three)."""
    import torch
    import paper_2509_19267_amd as rg
    from paper_2509_19267_amd import block_diagonal
    import workloads
    ps = workloads.laplacian_batch(count=count, n_min=2000, n_max=20000, seed=0)
    mats = []
    for p in ps:
        a = p.a.copy()
        a.data = a.data.astype(np.float32).astype(np.float64)
        mats.append(a)
    bs = [a @ p.x_star for a, p in zip(mats, ps)]
    rp, ci, v, ro, co = block_diagonal(mats)
    csr = (torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda(),
           torch.as_tensor(v).cuda())
    b = torch.as_tensor(np.concatenate(bs)).cuda()
    xs_np = np.concatenate([p.x_star for p in ps])
    xs = torch.as_tensor(xs_np).cuda()

    def timed(s, bb, xr):
        s.solve(bb, x_ref=xr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = s.solve(bb, x_ref=xr)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, x, info

    out = {"workload": f"laplacian_batch_{count}", "sum_n": int(sum(a.shape[1] for a in mats)),
           "tol": tol, "inner_tol": itol, "inner_max": imax}
    for form, c in [("fp64", csr), ("mixed_f32", (csr[0], csr[1], csr[2].to(torch.float32)))]:
        s = rg.BatchSolver(c, ro, co, eta=0.1, stop="err_ref", tol=tol,
                           max_iter=50000, inner_max=imax, inner_tol=itol,
                           precision=form)
        dt, x, info = timed(s, b, xs)
        s.close()
        err = float(np.linalg.norm(x.cpu().numpy() - xs_np) / np.linalg.norm(xs_np))
        out[f"{form}_batched_ms"] = round(1e3 * dt, 1)
        out[f"{form}_batched_iterations"] = int(info["iterations"])
        out[f"{form}_batched_converged"] = bool(info["converged"])
        out[f"{form}_batched_rel_err"] = err
        log(f"batched {form}: {1e3 * dt:.1f} ms, {info['iterations']} iterations")
    tot, its = 0.0, 0
    for a, bb, p in zip(mats, bs, ps):
        r0, c0, v0 = workloads.to_csr_arrays(a)
        s = rg.Solver(csr=(torch.as_tensor(r0).cuda(), torch.as_tensor(c0).cuda(),
                           torch.as_tensor(v0).cuda()), shape=a.shape, eta=0.1,
                      stop="err_ref", tol=tol, max_iter=50000, inner_max=imax,
                      inner_tol=itol)
        dt, x, info = timed(s, torch.as_tensor(bb).cuda(),
                            torch.as_tensor(p.x_star).cuda())
        s.close()
        tot += dt
        its += int(info["iterations"])
    out["fp64_one_by_one_ms"] = round(1e3 * tot, 1)
    out["fp64_one_by_one_iterations"] = its
    out["speedup_batched_fp64_vs_one_by_one"] = round(tot * 1e3 / out["fp64_batched_ms"], 3)
    out["speedup_batched_mixed_vs_one_by_one"] = round(tot * 1e3 / out["mixed_f32_batched_ms"], 3)
    log(f"one by one fp64: {1e3 * tot:.1f} ms")
    return out


def gdbek_vs_rgdbek(shapes=((8000, 500), (8000, 1000), (500, 8000),
                             (1000, 8000)), seeds=3, eta=0.5, tol=1e-6):
    """The comparison of Section 3 (Tables 1 and 2) on the same kernels:
    GDBEK's greedy sets vs RGDBEK's randomized draws (without replacement,
    and with replacement keeping the distinct indices), threshold / fraction
    eta = 0.5, stop at ||Ax - b||^2 <= tol ||b||^2, on sparse random matrices
    with 1% density (N(0,1) values, planted x*) -- synthetic stand-ins for
    the paper's sprandn matrices.  Mean iterations and time over `seeds`
    matrices per shape; the paper's mean iterations are quoted as context."""
    import torch
    import paper_2509_19267_amd as rg
    import workloads
    with open(os.path.join(ROOT, "tests", "golden", "paper_iteration_counts.json")) as f:
        gold = json.load(f)
    out = []
    for m, n in shapes:
        row = {"m": m, "n": n}
        for method in ["greedy", "random", "iid"]:
            its, ts = [], []
            for seed in range(seeds):
                p = workloads.sparse_uniform(m, n, density=0.01, seed=seed)
                rp, ci, v = workloads.to_csr_arrays(p.a)
                csr = (torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda(),
                       torch.as_tensor(v).cuda())
                s = rg.Solver(csr=csr, shape=(m, n), eta=eta, select=method,
                              stop="rse", tol=tol, max_iter=400_000, seed=seed)
                b = torch.as_tensor(p.b).cuda()
                s.solve(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = s.solve(b)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                its.append(info["iterations"])
                s.close()
            name = {"greedy": "gdbek", "random": "rgdbek",
                    "iid": "rgdbek_with_replacement"}[method]
            row[f"{name}_iterations"] = float(np.mean(its))
            row[f"{name}_ms"] = round(1e3 * float(np.mean(ts)), 2)
        key = ("tall_8000_rows", str(n)) if m == 8000 else ("fat_8000_columns", str(m))
        row["paper_rgdbek_iterations"] = gold[key[0]].get(key[1])
        row["paper_gdbek_iterations"] = gold["gdbek_" + key[0]].get(key[1])
        log(f"gdbek vs rgdbek {m}x{n}: {row}")
        out.append(row)
    return out


def differentiable_dense(m, n, tol=1e-10):
    """The differentiable form on the dense least-squares workload, FP64,
    block settings as tuned for the FP64 form, RES_EXT stop at tol (no
    reference solution inside a layer): time of the forward solve alone vs
    forward + backward (adjoint solve on A^T, second solve lam = A^+ w,
    gradient on A's m*n pattern), with the adjoint residual
    ||A^T w - dL/dx|| / ||dL/dx|| of the returned dL/db = w."""
    import torch
    import paper_2509_19267_amd as rg
    import workloads
    from paper_2509_19267_amd import tune
    prob = workloads.dense_least_squares(m, n, seed=0)
    ch = tune.lookup("dense", m, n, "fp64") or {}
    dev = torch.device("cuda", 0)
    a = torch.as_tensor(prob.a).to(dev)
    b = torch.as_tensor(prob.b).to(dev)
    st = torch.cuda.Stream()
    s = rg.Solver(a, k_col=ch.get("k_col", 0), k_row=ch.get("k_row", 0),
                  gram_aat=ch.get("gram_aat", False),
                  inner_tol=ch.get("inner_tol", 0.0),
                  inner_max=ch.get("inner_max", 0),
                  tile_rows=ch.get("tile_rows", 0), stop="res_ext", tol=tol,
                  max_iter=20000, stream=st)
    c = torch.randn(n, dtype=torch.float64, device=dev)
    values = a.reshape(-1).detach().requires_grad_(True)

    def fwd():
        x, info = s.solve(b)
        torch.cuda.synchronize()
        return info

    def fwd_bwd():
        bt = b.clone().requires_grad_(True)
        x = rg.solve(s, values, bt, least_squares=True)
        (x * c).sum().backward()
        torch.cuda.synchronize()
        return bt.grad

    fwd()
    fwd_bwd()
    values.grad = None
    t0 = time.perf_counter()
    info = fwd()
    t_f = time.perf_counter() - t0
    t0 = time.perf_counter()
    w = fwd_bwd()
    t_fb = time.perf_counter() - t0
    adj = float(torch.linalg.norm(a.t() @ w - c) / torch.linalg.norm(c))
    out = {"workload": f"dense_least_squares_{m}x{n}", "stop": "res_ext",
           "tol": tol, "forward_iterations": info["iterations"],
           "forward_ms": round(1e3 * t_f, 2),
           "forward_backward_ms": round(1e3 * t_fb, 2),
           "backward_over_forward": round((t_fb - t_f) / t_f, 3),
           "adjoint_residual": adj,
           "grad_A_finite": bool(torch.isfinite(values.grad).all())}
    s.close()
    log(f"differentiable: {out}")
    return out


def fem_table8(max_iter=10000, eta=0.5, tol=1e-6):
    """Section 6's finite-element systems at the paper's settings (eta = 0.5,
    stop at ||Ax - b||^2 <= tol ||b||^2 or after max_iter iterations):
    Poisson on 25 x 25 nodes, Helmholtz k = 25 on 50 x 50 nodes, P1
    triangles.  Reports iterations, time, the RSE reached and the relative
    nodal L2 error against the exact solution, beside Table 8's figures."""
    import torch
    import paper_2509_19267_amd as rg
    import workloads
    with open(os.path.join(ROOT, "tests", "golden", "paper_fem_table8.json")) as f:
        gold = json.load(f)
    out = {}
    for name, (npts, k, mode) in (("poisson", (25, 0.0, 1)),
                                  ("helmholtz", (50, 25.0, 4))):
        A, b, u, _ = workloads.fem_p1_unit_square(npts, k, mode)
        rp, ci, v = workloads.to_csr_arrays(A)
        csr = (torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda(),
               torch.as_tensor(v).cuda())
        s = rg.Solver(csr=csr, shape=A.shape, eta=eta, stop="rse", tol=tol,
                      max_iter=max_iter)
        bt = torch.as_tensor(b).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = s.solve(bt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s.close()
        xh = x.cpu().numpy()
        row = {"n": int(A.shape[0]), "nnz": int(A.nnz),
               "iterations": info["iterations"],
               "converged": bool(info["converged"]),
               "ms": round(1e3 * el, 1),
               "us_per_iteration": round(1e6 * el / max(info["iterations"], 1), 1),
               "rse": float(np.linalg.norm(b - A @ xh) ** 2 / np.linalg.norm(b) ** 2),
               "rel_l2": float(np.linalg.norm(xh - u) / np.linalg.norm(u)),
               "paper_rse": gold[name]["rse"],
               "paper_rel_l2": gold[name]["rel_l2"]}
        log(f"fem {name}: {row}")
        out[name] = row
    return out


def cpu_baseline(prob, choice, gpu_iters, budget_s=20.0):
    """The FP64 oracle on the host cores: a bounded sample of full-size
    iterations (same block sizes), scaled to the iterations the FP64 GPU path
    needed to reach the tolerance."""
    from oracle.rgdbek import rgdbek
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    it = 0
    t0 = time.perf_counter()
    x, z = None, None
    while True:
        x, z, _ = rgdbek(prob.a, prob.b, k_col=choice["k_col"],
                         k_row=choice["k_row"], max_iter=1, seed=0,
                         x0=x, z0=z, it0=it)
        it += 1
        el = time.perf_counter() - t0
        if el > budget_s or it >= 50:
            break
    per_it = el / it
    return {"value": round(per_it * gpu_iters * 1e3, 1), "unit": "ms",
            "cores": int(cores), "kind": "oracle",
            "sample": f"{it} full-size oracle iterations ({el:.1f} s, "
                      f"{per_it*1e3:.0f} ms each) scaled to the {gpu_iters} "
                      f"iterations of the FP64 GPU solve"}


if __name__ == "__main__":
    main()
