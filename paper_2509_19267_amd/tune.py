"""Block-size autotuner.

RGDBEK's block fraction trades per-iteration cost against iteration count
(the remark on eta in Section 2), and the inner tolerance of the block
projections trades inner steps against outer progress.  The tuner times
real solves to the target tolerance on the problem at hand over a grid of
(k_col, k_row), then over the inner tolerance and step cap, and keeps the
fastest converging choice; the row-tile height of the dense residual pass
is then picked by timing that pass alone (its effect on a whole solve is
within run-to-run noise), and the choice is checked to converge.  Results
are cached per (layout, m, n, form) in tuned.json next to this file.
"""
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _key(layout, m, n, form):
    return f"{layout}:{m}x{n}:{form}"


def lookup(layout, m, n, form="fp64"):
    return _load().get(_key(layout, m, n, form))


def store(layout, m, n, form, choice):
    c = _load()
    c[_key(layout, m, n, form)] = choice
    try:
        with open(CACHE, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    except OSError:
        pass


def _time_solve(a, b, x_ref, choice, *, stream, tol, precision, reps,
                with_create=False):
    import torch
    from .solver import Solver
    torch.cuda.synchronize()
    tc = time.perf_counter()
    s = Solver(a, k_col=choice["k_col"], k_row=choice["k_row"],
               gram_aat=choice.get("gram_aat", False), stop="err_ref",
               tol=tol, max_iter=5000, precision=precision, stream=stream,
               inner_tol=choice.get("inner_tol", 0.0),
               inner_max=choice.get("inner_max", 0),
               tile_rows=choice.get("tile_rows", 0),
               pass_drop=choice.get("pass_drop", 0.0))
    torch.cuda.synchronize()
    create = time.perf_counter() - tc
    ts, ok, its = [], True, 0
    try:
        for _ in range(reps):
            t0 = time.perf_counter()
            _, info = s.solve(b, x_ref=x_ref)
            ts.append(time.perf_counter() - t0)
            ok = ok and bool(info["converged"])
            its = info["iterations"]
    finally:
        s.close()
    if with_create:
        return min(ts), ok, its, create
    return min(ts), ok, its


def _time_pass(a, tile_rows, precision, stream, reps=30, rounds=3):
    """Mean time of one fused residual pass (rgdbek_apply) with the given
    row tile, best of `rounds` rounds of `reps` launches, timed with events
    on the handle's stream."""
    import torch
    from .solver import Solver
    m, n = a.shape
    prec = "f32" if precision == "mixed_f32" else "f64"
    dt = torch.float32 if prec == "f32" else torch.float64
    s = Solver(a, k_col=8, k_row=8, precision="mixed_f32", stream=stream,
               tile_rows=tile_rows)
    try:
        xv = torch.randn(n, dtype=dt, device=a.device)
        zv = torch.randn(m, dtype=dt, device=a.device)
        ax = torch.empty(m, dtype=dt, device=a.device)
        atz = torch.empty(n, dtype=dt, device=a.device)
        st = stream if stream is not None else torch.cuda.current_stream()
        for _ in range(3):
            s.apply(xv, zv, ax, atz, precision=prec)
        best = float("inf")
        for _ in range(rounds):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(reps):
                s.apply(xv, zv, ax, atz, precision=prec)
            e1.record(st)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / reps)
    finally:
        s.close()
    return best


def tune_dense(a, b, x_ref, *, stream=None, tol=1e-8, log=print,
               precision="fp64", reps=2):
    """Sweep the block sizes, the inner tolerance and step cap, the mixed
    form's pass drop, and the row tile of the fused pass for a dense A
    (device tensors) in one arithmetic form; returns and caches the fastest
    converging choice, with the precomputed A A^T weighed against its set-up
    cost.  The benchmark tunes on another draw of its workload (generator
    seed 1) than the one it times."""
    m, n = a.shape

    def run(ch, best):
        try:
            t, ok, its = _time_solve(a, b, x_ref, ch, stream=stream, tol=tol,
                                     precision=precision, reps=reps)
        except Exception as e:  # noqa: BLE001
            log(f"tune {precision} {ch}: failed: {e}")
            return best
        log(f"tune {precision} {ch}: {1e3 * t:.1f} ms ({its} it, "
            f"converged={ok})")
        if ok and (best is None or t < best[0]):
            return (t, dict(ch))
        return best

    best = None
    # fractions of n for both blocks, below 1 (the sampling parameter of
    # Theorem 2.3 lies in (0, 1); row blocks of up to n rows keep the Gram
    # form); large blocks pay off on tall systems
    for fc in [0.2, 0.4, 0.6, 0.8, 0.9]:
        for fr in [0.2, 0.4, 0.6, 0.8, 0.9]:
            kc = max(1, min(int(fc * n), n))
            kr = max(1, min(int(fr * n), m))
            best = run(dict(k_col=kc, k_row=kr, gram_aat=kr > 256,
                            inner_tol=0.1, inner_max=16), best)
    if best is None:
        raise RuntimeError("no configuration converged")
    base = best[1]
    for itol in [0.3, 0.1, 0.03, 0.01, 1e-3]:
        for imax in [4, 8, 16, 32]:
            ch = dict(base, inner_tol=itol, inner_max=imax)
            if ch != base:
                best = run(ch, best)
    base = best[1]
    if precision == "mixed_f32":
        # residual drop that ends a refinement pass
        for pd in [1e-3, 1e-4, 1e-5]:
            best = run(dict(base, pass_drop=pd), best)
        base = best[1]
    times = {}
    for tr in [0, 64, 128, 160, 224, 256, 320, 400]:
        times[tr] = _time_pass(a, tr, precision, stream)
        log(f"tune {precision} fused pass tile_rows={tr}: "
            f"{1e3 * times[tr]:.1f} us")
    tr = min(times, key=times.get)
    chosen = run(dict(base, tile_rows=tr), None)
    if chosen is None:
        chosen = best
    # the precomputed A A^T against its set-up cost: solve time alone picks
    # the choice (the benchmark times solves), and the create-inclusive cost
    # of one solve per handle is recorded for both settings
    ch = dict(chosen[1])
    costs = {}
    for g in (True, False):
        try:
            t, ok, its, c = _time_solve(a, b, x_ref, dict(ch, gram_aat=g),
                                        stream=stream, tol=tol,
                                        precision=precision, reps=reps,
                                        with_create=True)
        except Exception as e:  # noqa: BLE001
            log(f"tune {precision} gram_aat={g}: failed: {e}")
            continue
        log(f"tune {precision} gram_aat={g}: solve {1e3 * t:.1f} ms, "
            f"create {1e3 * c:.1f} ms")
        if ok:
            costs[g] = (t, c)
    if costs:
        g_best = min(costs, key=lambda g: costs[g][0])
        ch["gram_aat"] = g_best
        ch["solve_ms"] = round(1e3 * costs[g_best][0], 2)
        ch["create_ms"] = round(1e3 * costs[g_best][1], 1)
        ch["create_plus_one_solve_ms"] = {
            str(g).lower(): round(1e3 * (t + c), 1) for g, (t, c) in costs.items()}
    store("dense", m, n, precision, ch)
    return ch


# block fractions the sparse tuner may extend its grid to, in order
ETA_LADDER = (0.05, 0.1, 0.2, 0.3, 0.5, 0.7, 1.0)


def next_eta(eta):
    """The ladder's next block fraction above eta (None at the top)."""
    for e in ETA_LADDER:
        if e > eta + 1e-12:
            return e
    return None


def tune_sparse(make, b, x_ref, *, key, tol=1e-8, log=print, reps=1,
                etas=(0.05, 0.1, 0.2),
                inner=((0.5, 2), (0.3, 4), (0.1, 8), (0.1, 16), (0.03, 16)),
                graph_iters=(4, 8, 16), pass_drops=(), extend=False):
    """Tune a sparse solve (single system, batch or many right-hand sides):
    `make(eta=, inner_tol=, inner_max=, graph_iters=[, pass_drop=])` builds a
    handle (the caller picks its stop test and tol); each setting is timed
    over `reps` solves after one warm-up solve (graph capture).  Block
    fraction and inner settings first -- with `extend`, while the largest
    block fraction tried is the fastest, the next one of ETA_LADDER is tried
    too -- then the iterations per captured graph, then (for the mixed form)
    the drop that ends a refinement pass, each at the best of the earlier
    stages; the fastest converging choice is cached under `key` and
    returned."""
    import torch

    def sync():
        if torch.cuda.is_available():
            torch.cuda.synchronize()

    def run(ch, best):
        try:
            s = make(**ch)
        except Exception as e:  # noqa: BLE001
            log(f"tune {key} {ch}: failed: {e}")
            return best
        try:
            s.solve(b, x_ref=x_ref)
            ts, ok, its = [], True, 0
            for _ in range(reps):
                sync()
                t0 = time.perf_counter()
                _, info = s.solve(b, x_ref=x_ref)
                sync()
                ts.append(time.perf_counter() - t0)
                ok = ok and bool(info["converged"])
                its = info["iterations"]
        finally:
            s.close()
        t = min(ts)
        log(f"tune {key} {ch}: {1e3 * t:.1f} ms ({its} it, converged={ok})")
        if ok and (best is None or t < best[0]):
            return (t, dict(ch, solve_ms=round(1e3 * t, 2), iterations=its))
        return best

    best = None
    tried = []

    def sweep(eta, best):
        tried.append(eta)
        for itol, imax in inner:
            best = run(dict(eta=eta, inner_tol=itol, inner_max=imax,
                            graph_iters=8), best)
        return best

    for eta in etas:
        best = sweep(eta, best)
    while extend and best is not None and best[1]["eta"] >= max(tried):
        nxt = next_eta(max(tried))
        if nxt is None:
            break
        best = sweep(nxt, best)
    if best is None:
        raise RuntimeError(f"no configuration of {key} converged")
    best[1]["etas_tried"] = sorted(tried)
    base = {k: best[1][k] for k in ("eta", "inner_tol", "inner_max")}
    for gi in graph_iters:
        if gi != 8:
            best = run(dict(base, graph_iters=gi), best)
    best[1]["etas_tried"] = sorted(tried)
    if pass_drops:
        base = {k: best[1][k] for k in ("eta", "inner_tol", "inner_max",
                                        "graph_iters")}
        for pd in pass_drops:
            best = run(dict(base, pass_drop=pd), best)
    best[1]["etas_tried"] = sorted(tried)
    c = _load()
    c[key] = best[1]
    try:
        with open(CACHE, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return best[1]
