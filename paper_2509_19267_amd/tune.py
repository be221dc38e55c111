"""Block-size autotuner.

RGDBEK's block fraction trades per-iteration cost against iteration count
(the remark on eta in Section 2).  The tuner times real solves on the
problem at hand over a small grid of (k_col, k_row) and dense Gram options
and keeps the fastest time-to-tolerance.  Results are cached per
(layout, m, n) in tuned.json next to this file.
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


def lookup(layout, m, n):
    return _load().get(f"{layout}:{m}x{n}")


def store(layout, m, n, choice):
    c = _load()
    c[f"{layout}:{m}x{n}"] = choice
    try:
        with open(CACHE, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    except OSError:
        pass


def _time_solve(a, b, x_ref, choice, *, stream, tol, precision, reps):
    from .solver import Solver
    s = Solver(a, k_col=choice["k_col"], k_row=choice["k_row"],
               gram_aat=choice.get("gram_aat", False), stop="err_ref",
               tol=tol, max_iter=5000, precision=precision, stream=stream,
               inner_tol=choice.get("inner_tol", 0.0),
               inner_max=choice.get("inner_max", 0))
    ts, ok, its = [], True, 0
    for _ in range(reps):
        t0 = time.perf_counter()
        _, info = s.solve(b, x_ref=x_ref)
        ts.append(time.perf_counter() - t0)
        ok = ok and bool(info["converged"])
        its = info["iterations"]
    s.close()
    return min(ts), ok, its


def tune_dense(a, b, x_ref, *, stream=None, tol=1e-8, log=print,
               grid=None, precision="fp64", reps=2):
    """Sweep block sizes (k_col, k_row, A A^T precomputed or not), then the
    inner CG tolerance and step cap, for a dense A (device tensors); returns
    and caches the fastest converging choice."""
    m, n = a.shape
    if grid is None:
        fr = [0.02, 0.05, 0.1, 0.2]
        grid = []
        for fc in fr:
            for frw in fr:
                kc = max(1, int(fc * n))
                kr = max(1, min(int(frw * n), m))
                grid.append(dict(k_col=kc, k_row=kr, gram_aat=kr > 256,
                                 inner_tol=1e-10, inner_max=48))
    best = None
    for ch in grid:
        try:
            t, ok, its = _time_solve(a, b, x_ref, ch, stream=stream, tol=tol,
                                     precision=precision, reps=reps)
        except Exception as e:  # noqa: BLE001
            log(f"tune {ch}: failed: {e}")
            continue
        log(f"tune {ch}: {1e3*t:.1f} ms ({its} it, converged={ok})")
        if ok and (best is None or t < best[0]):
            best = (t, ch)
    if best is None:
        raise RuntimeError("no configuration converged")
    base = best[1]
    for itol in [1e-14, 1e-10, 1e-8, 1e-6]:
        for imax in [16, 24, 32, 48, 64]:
            ch = dict(base, inner_tol=itol, inner_max=imax)
            if ch == base:
                continue
            try:
                t, ok, its = _time_solve(a, b, x_ref, ch, stream=stream,
                                         tol=tol, precision=precision,
                                         reps=reps)
            except Exception as e:  # noqa: BLE001
                log(f"tune {ch}: failed: {e}")
                continue
            log(f"tune {ch}: {1e3*t:.1f} ms ({its} it, converged={ok})")
            if ok and t < best[0]:
                best = (t, ch)
    store("dense", m, n, best[1])
    return best[1]
