"""Resolution study of Figure 1 (Section 2 numerical example) on the GPU path.

Disk of radius pi/15 centred in the unit square, E_inclusion / E_matrix =
1e3 and 1e-3 (nu = 0.3), mean axial stress under a 1 % uniaxial strain
(linear, so C_1111 carries it), fixed-point tolerance 1e-4, FP64.  Each
treatment -- no filter (indicator at the pixel centre), or the Voigt,
Reuss and 2-layer filters at several radii (pixel units) -- is solved at
the 25 odd resolutions from 7 to 125 whose prime factors are at most 13.  N_1% is the smallest swept
resolution from which every finer swept resolution is within 1 % of the
converged stress, taken as the median of the four treatments at radius 0.55
on a 243 x 243 grid.  Section 2 reports, for the two efficient filters of
each contrast, an optimum radius of 0.5-0.55 at which N_1% is divided by
2.6 to 7.2.  Checked here: for each contrast the filter with the smallest
N_1% reaches it at radius 0.55 (of 0.3, 0.55, 1, 1.5), and the unfiltered
N_1% over that one lies in the printed 2.6-7.2 range.  The swept sizes are
sparser than the paper's (every size from 6 to 128: the transforms need
prime factors of at most 13); the whole table is printed.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import log
from workloads import FIG1_RESOLUTIONS, fig1_disk_case

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CONTRASTS = (1e3, 1e-3)
RULES = ("voigt", "reuss", "laminate")
RADII = (0.3, 0.55, 1.0, 1.5)
REF_N = 243


@pytest.fixture(scope="module")
def hm():
    import paper_1412_3228_amd as hm_mod
    assert torch.cuda.is_available() and hm_mod.device_ok()
    return hm_mod


def _problem(hm, w):
    _, frac, incl = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, "fp64", DEV)
    return {"n": w.n, "dim": 2, "phases": w.phases, "rule": w.rule, "frac": frac, "incl": incl,
            "spheres": w.spheres}


def n_one_percent(stress_by_n, ref):
    """Smallest swept n from which every finer swept n is within 1 % of ref (None if the finest is not)."""
    best = None
    for n in sorted(stress_by_n, reverse=True):
        if abs(stress_by_n[n] / ref - 1.0) <= 0.01:
            best = n
        else:
            break
    return best


def test_fig1_resolution_study(hm):
    treatments = [("none", 0.0)] + [(rule, r) for rule in RULES for r in RADII]
    keys, probs = [], []
    for c in CONTRASTS:
        for n in FIG1_RESOLUTIONS:
            for rule, r in treatments:
                keys.append((c, rule, r, n))
                probs.append(_problem(hm, fig1_disk_case(n, c, rule, r if r > 0 else 1.0)))
        for rule in ("none",) + RULES:
            keys.append((c, rule, -1.0, REF_N))
            probs.append(_problem(hm, fig1_disk_case(REF_N, c, rule, 0.55)))
    log("fig1 study: %d cells" % len(probs))
    out = hm.hm_effective_tensor_batch(probs, prec="fp64", tol=1e-4, max_iter=30000, check_every=32)
    stress, iters = {}, {}
    for k, res in zip(keys, out["results"]):
        assert all(rep["status"] == 0 for rep in res["reports"]), (k, res["reports"])
        stress[k] = 0.01 * res["C"][0, 0]  # <sigma_11> under eps_11 = 1 %
        iters[k] = res["reports"][0]["iters"]
    factors = {}
    for c in CONTRASTS:
        ref = float(np.median([stress[(c, rule, -1.0, REF_N)] for rule in ("none",) + RULES]))
        rows = {}
        for rule, r in treatments:
            rows[(rule, r)] = n_one_percent({n: stress[(c, rule, r, n)] for n in FIG1_RESOLUTIONS}, ref)
        log("contrast %g: converged <sigma_11> = %.6g" % (c, ref))
        for (rule, r), v in rows.items():
            curve = " ".join("%.4f" % (stress[(c, rule, r, n)] / ref) for n in FIG1_RESOLUTIONS)
            log("  %-8s r=%-4g N1%%=%-5s  ratios %s" % (rule, r, v, curve))
        n_none = rows[("none", 0.0)]
        assert n_none is not None
        finite = {k: v for k, v in rows.items() if k[0] != "none" and v is not None}
        best_rule, best_r = min(finite, key=lambda k: (finite[k], k[1]))
        factors[c] = n_none / finite[(best_rule, best_r)]
        its = {rule: iters[(c, rule, 0.55 if rule != "none" else 0.0, FIG1_RESOLUTIONS[-1])]
               for rule in ("none",) + RULES}
        log("  best: %s r=%g N1%%=%d, unfiltered N1%%=%d, factor %.2f (problem size / %.1f); iterations at "
            "n=%d, r=0.55: %s" % (best_rule, best_r, finite[(best_rule, best_r)], n_none, factors[c],
                                  factors[c] ** 2, FIG1_RESOLUTIONS[-1], its))
        assert best_r == 0.55
        assert 2.6 <= factors[c] <= 7.2
