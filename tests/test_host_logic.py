"""Host-side logic that needs no GPU: the tuner cache, the benchmark's
traffic lookup against the committed counter summary, and its argument
defaults."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2509_19267_amd import tune  # noqa: E402


def test_tuned_choices_are_complete():
    for form in ("fp64", "mixed_f32"):
        ch = tune.lookup("dense", 20000, 5000, form)
        assert ch is not None, form
        for key in ("k_col", "k_row", "inner_tol", "inner_max", "tile_rows"):
            assert key in ch, (form, key)
        assert 0 < ch["k_col"] <= 5000 and 0 < ch["k_row"] <= 5000


def test_counted_traffic_matches_the_tuned_tiles():
    # the committed counter summary is for the tuned row tiles: the
    # benchmark's roofline then carries measured traffic, not null
    for form, prec in (("fp64", "f64"), ("mixed_f32", "f32")):
        tr = tune.lookup("dense", 20000, 5000, form)["tile_rows"]
        t = bench.counted_traffic(prec, tr, 20000, 5000)
        assert isinstance(t, int), (form, tr)
        alg = 20000 * 5000 * (8 if prec == "f64" else 4)
        assert alg <= t <= 1.1 * alg
    assert bench.counted_traffic("f32", 12345, 20000, 5000) is None
    assert bench.counted_traffic("f32", 224, 1000, 500) is None


def test_tune_cache_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "t.json"))
    assert tune.lookup("dense", 3, 4, "fp64") is None
    tune.store("dense", 3, 4, "fp64", {"k_col": 2, "k_row": 3})
    tune.store("dense", 3, 4, "mixed_f32", {"k_col": 1, "k_row": 1})
    assert tune.lookup("dense", 3, 4, "fp64") == {"k_col": 2, "k_row": 3}
    data = json.load(open(tmp_path / "t.json"))
    assert set(data) == {"dense:3x4:fp64", "dense:3x4:mixed_f32"}


def test_bench_defaults(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert a.gpus == 1 and a.steps >= 1 and a.warmup >= 0
    assert (a.m, a.n, a.tol) == (20000, 5000, 1e-8)


def test_deblur_cpu_leg_checks_against_closed_form():
    # the deblurring workload's CPU leg compares solutions and gradients
    # with the Kronecker closed forms: fed the dense least-squares solutions
    # and the dense pinv gradients of a 16 x 16 instance it must report
    # agreement to rounding
    import numpy as np
    import workloads
    from oracle.refsol import grad_reference
    aug, t, s = workloads.blur_tikhonov(npix=16, mu=1e-2)
    n, nrhs = 256, 2
    rng = np.random.default_rng(0)
    b_img = rng.standard_normal((n, nrhs))
    cs = rng.standard_normal((nrhs, n))
    ad = aug.toarray()
    ac = aug.tocsr()
    ac.sort_indices()
    rows = np.repeat(np.arange(ac.shape[0]), np.diff(ac.indptr))
    xs, dbs, dv = [], [], np.zeros(aug.nnz)
    for r in range(nrhs):
        bb = np.concatenate([b_img[:, r], np.zeros(n)])
        xs.append(np.linalg.lstsq(ad, bb, rcond=None)[0])
        da, w = grad_reference(ad, bb, cs[r])
        dbs.append(w)
        dv += da[rows, ac.indices]
    ctx = {"c4": {"t": t, "s": s, "b_img": b_img,
                  "sols": {"fp64": np.array(xs).T}, "aug": aug,
                  "grads": {"x": np.array(xs).T, "db": np.array(dbs).T,
                            "dv": dv, "c": cs.T}}}
    out = bench.cpu_baseline_full(["c4"], ctx, budget_s=0.2)
    assert out["c4_rel_err_vs_closed_form_max"]["fp64"] <= 1e-10
    g = out["c4_differentiable_vs_closed_form"]
    assert g["x_rel_err_max"] <= 1e-10
    assert g["db_rel_err"] <= 1e-10
    assert g["dA_sampled_rel_err"] <= 1e-10
    assert out["c4"]["iterations"] >= 1


def test_sparse_tuner_extends_its_block_fraction_grid(tmp_path, monkeypatch):
    # a stand-in handle whose solve time is smallest at eta = 0.7: started
    # on (0.2, 0.3, 0.5), the tuner must climb the ladder to 0.7, try 1.0,
    # and keep 0.7; without `extend` it stops at the grid's edge
    import time as _time
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "t.json"))

    class Fake:
        def __init__(self, eta, inner_tol, inner_max, graph_iters, **_):
            self.eta = eta

        def solve(self, b, x_ref=None):
            _time.sleep(0.002 + 0.01 * abs(self.eta - 0.7))
            return None, {"converged": True, "iterations": 10}

        def close(self):
            pass

    got = tune.tune_sparse(Fake, None, None, key="fake", log=lambda *_: None,
                           etas=(0.2, 0.3, 0.5), graph_iters=(8,),
                           extend=True)
    assert got["eta"] == 0.7
    assert got["etas_tried"] == [0.2, 0.3, 0.5, 0.7, 1.0]
    got = tune.tune_sparse(Fake, None, None, key="fake2", log=lambda *_: None,
                           etas=(0.2, 0.3, 0.5), graph_iters=(8,))
    assert got["eta"] == 0.5 and got["etas_tried"] == [0.2, 0.3, 0.5]
    assert tune.next_eta(1.0) is None and tune.next_eta(0.5) == 0.7
