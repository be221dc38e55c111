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


def tune_dense(a, b, x_ref, *, stream=None, tol=1e-8, log=print,
               grid=None, precision="fp64", reps=2):
    """Sweep (k_col, k_row, gram_aat) for a dense A (device tensors);
    returns and caches the fastest choice."""
    from .solver import Solver
    m, n = a.shape
    if grid is None:
        fr = [0.02, 0.05, 0.1, 0.2]
        grid = []
        for fc in fr:
            for frw in fr:
                kc = max(1, int(fc * n))
                kr = max(1, min(int(frw * n), m))
                grid.append((kc, kr, kr > 256))
    best = None
    for kc, kr, aat in grid:
        try:
            s = Solver(a, k_col=kc, k_row=kr, gram_aat=aat, stop="err_ref",
                       tol=tol, max_iter=5000, precision=precision,
                       stream=stream)
        except Exception as e:  # noqa: BLE001
            log(f"tune {kc},{kr},{aat}: create failed: {e}")
            continue
        ts = []
        ok = True
        for _ in range(reps):
            t0 = time.perf_counter()
            _, info = s.solve(b, x_ref=x_ref)
            ts.append(time.perf_counter() - t0)
            ok = ok and bool(info["converged"])
        s.close()
        t = min(ts)
        log(f"tune k_col={kc} k_row={kr} gram_aat={aat}: {1e3*t:.1f} ms "
            f"({info['iterations']} it, converged={ok})")
        if ok and (best is None or t < best[0]):
            best = (t, dict(k_col=kc, k_row=kr, gram_aat=aat))
    if best is None:
        raise RuntimeError("no configuration converged")
    store("dense", m, n, best[1])
    return best[1]
