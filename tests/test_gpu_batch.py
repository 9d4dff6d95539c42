"""GPU tests of the batched solve of many cells of uneven sizes."""
import numpy as np
import pytest
import torch

from gpu_helpers import log, rel
from workloads import small_sphere_case, workload_c4

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def hm():
    import paper_1412_3228_amd as hm_mod
    assert torch.cuda.is_available() and hm_mod.device_ok()
    return hm_mod


def _prob(hm, w, prec):
    cnt, frac, incl = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, prec, DEV)
    return {"n": w.n, "dim": w.dim, "phases": w.phases, "rule": w.rule, "frac": frac, "incl": incl,
            "spheres": w.spheres}


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_single_cell_solves(hm, use_graph):
    cases = [small_sphere_case(n=(15, 15, 15), contrast=10.0, rule="laminate", subsamples=4),
             small_sphere_case(n=(21, 21, 21), contrast=0.05, rule="reuss", subsamples=4),
             small_sphere_case(n=(15, 15, 15), contrast=30.0, rule="voigt", subsamples=4, offset=(1.0, 0.5, 0.0)),
             small_sphere_case(n=(27, 27, 1), dim=2, contrast=5.0, rule="laminate", subsamples=8),
             small_sphere_case(n=(21, 21, 21), contrast=3.0, rule="laminate", subsamples=4)]
    log("batch of %d cells (graph %s)" % (len(cases), use_graph))
    probs = [_prob(hm, w, "fp64") for w in cases]
    kw = dict(prec="fp64", tol=1e-8, max_iter=3000, check_every=8, autotune=False)
    out = hm.hm_effective_tensor_batch(probs, use_graph=use_graph, **kw)
    for w, pr, res in zip(cases, probs, out["results"]):
        single = hm.hm_effective_tensor(w.n, w.dim, w.phases, w.rule, pr["frac"], pr["incl"], w.spheres, **kw)
        assert np.array_equal(res["C"], single["C"])
        assert [r["iters"] for r in res["reports"]] == [r["iters"] for r in single["reports"]]


def test_c4_batch_of_64_uneven_cells_mixed(hm):
    works = workload_c4()
    log("c4: %d cells, sizes %s" % (len(works), sorted(set(w.n[0] for w in works))))
    probs = [_prob(hm, w, "mixed") for w in works]
    out = hm.hm_effective_tensor_batch(probs, prec="mixed", tol=1e-4, max_iter=4000, check_every=16,
                                       stall_window=20, use_graph=True)
    its = [max(r["iters"] for r in res["reports"]) for res in out["results"]]
    log("c4 iterations min %d max %d" % (min(its), max(its)))
    assert all(r["status"] in (0, 2) for res in out["results"] for r in res["reports"])
    # sampled cells against FP64 single-cell solves
    for i in (0, 17, 41, 63):
        w = works[i]
        p64 = _prob(hm, w, "fp64")
        ref = hm.hm_effective_tensor(w.n, w.dim, w.phases, w.rule, p64["frac"], p64["incl"], w.spheres,
                                     prec="fp64", tol=1e-9, max_iter=20000, check_every=32, use_graph=True)
        e = rel(out["results"][i]["C"], ref["C"])
        log("c4 cell %d (n=%d, contrast %.3g): mixed batch vs fp64 %.2e" % (i, w.n[0], w.meta["contrast"], e))
        assert e < 1e-5
