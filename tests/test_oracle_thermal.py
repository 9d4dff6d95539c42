"""Pins of the conductivity oracle (the scalar counterpart of Section 2's
scheme): rule closed forms and Wiener ordering, exact layered cells,
Hashin-Shtrikman bounds and isotropy for the centred sphere, the dense
direct solve, and the 2D antiplane-shear analogy with the elastic oracle."""
import numpy as np
import pytest

from oracle import filter as F, rules, solver, thermal as T
from workloads import lame, small_sphere_case

K = (1.0, 10.0)


def test_rules_closed_forms_and_wiener_order():
    n = np.array([0.6, 0.0, 0.8])
    for f in (0.0, 0.3, 0.71, 1.0):
        a = (1 - f) * K[0] + f * K[1]
        h = 1.0 / ((1 - f) / K[0] + f / K[1])
        assert np.allclose(T.rule_tensor("voigt", f, n, K), a * np.eye(3))
        assert np.allclose(T.rule_tensor("reuss", f, n, K), h * np.eye(3))
        L = T.rule_tensor("laminate", f, n, K)
        ev = np.sort(np.linalg.eigvalsh(L))
        assert np.allclose(ev, np.sort([h, a, a]))
        assert np.allclose(L @ n, h * n)  # the normal sees the layers in series
        assert h <= a + 1e-15


def _layered(n, rows):
    """Pure-voxel layers normal to x: rows[x] is 0 (matrix) or 1 (inclusion)."""
    frac = np.zeros((n[2], n[1], n[0]))
    frac[:, :, :] = np.asarray(rows, dtype=np.float64)[None, None, :]
    return frac.reshape(-1)


def test_grid_aligned_layers_are_exact():
    n = (9, 5, 3)
    rows = [0, 1, 1, 0, 0, 1, 0, 0, 0]
    f = np.mean(rows)
    fld = T.ConductivityField(n, 3, K, "none", _layered(n, rows))
    Kt, reps = T.effective_conductivity(fld, T.reference_conductivity(K), 1e-12, 20000, 3)
    harm = 1.0 / ((1 - f) / K[0] + f / K[1])
    arith = (1 - f) * K[0] + f * K[1]
    assert np.allclose(np.diag(Kt), [harm, arith, arith], rtol=1e-9)
    assert np.allclose(Kt - np.diag(np.diag(Kt)), 0.0, atol=1e-10)


def test_sphere_cell_bounds_and_rule_order():
    # Effective conductivity is monotone in the local tensors and pointwise
    # harmonic I <= laminate <= arithmetic I, so K_reuss <= K_laminate <=
    # K_voigt.  Pure-voxel and laminate cells are realisable two-phase
    # composites (a laminate voxel is a rank-one layering of the two phases),
    # so they obey the Hashin-Shtrikman bounds at the inclusion fraction;
    # every rule obeys the Wiener bounds of its own voxel tensors.
    w = small_sphere_case(n=(9, 9, 9), contrast=10.0, rule="laminate", radius_vox=1.0, subsamples=4)
    ff = F.filter_field(w)
    nrm = F.interface_normals(w.n, 3, w.spheres, ff["incl"], F.all_voxels(w.n))
    f = ff["frac"].mean()
    k1, k2 = K
    lo = k1 + f / (1.0 / (k2 - k1) + (1 - f) / (3 * k1))
    hi = k2 + (1 - f) / (1.0 / (k1 - k2) + f / (3 * k2))
    got = {}
    for rule in ("none", "voigt", "reuss", "laminate"):
        frac = (ff["frac"] >= 0.5).astype(np.float64) if rule == "none" else ff["frac"]
        fld = T.ConductivityField(w.n, 3, K, rule, frac, nrm if rule == "laminate" else None)
        Kt, reps = T.effective_conductivity(fld, T.reference_conductivity(K), 1e-10, 5000, 3)
        assert all(r["status"] == T.STATUS_CONVERGED for r in reps)
        kk = Kt[0, 0]
        assert np.allclose(Kt, kk * np.eye(3), rtol=1e-8, atol=1e-10)  # cubic symmetry
        vk = np.array([T.rule_tensor(rule if rule != "none" else "voigt", fi, np.array([1.0, 0, 0]), K)[1, 1]
                       for fi in frac])
        harm = 1.0 / np.mean(1.0 / vk) if rule != "laminate" else 1.0 / ((1 - f) / k1 + f / k2)
        arith = np.mean(vk) if rule != "laminate" else (1 - f) * k1 + f * k2
        assert harm - 1e-12 <= kk <= arith + 1e-12
        got[rule] = kk
    for rule in ("none", "laminate"):
        fr = np.mean((ff["frac"] >= 0.5)) if rule == "none" else f
        lo_r = k1 + fr / (1.0 / (k2 - k1) + (1 - fr) / (3 * k1))
        hi_r = k2 + (1 - fr) / (1.0 / (k1 - k2) + fr / (3 * k2))
        assert lo_r - 1e-9 <= got[rule] <= hi_r + 1e-9
    assert got["reuss"] <= got["laminate"] <= got["voigt"]
    assert lo < got["laminate"] < hi


def test_homogeneous_cell_converges_at_once():
    n = (5, 7, 3)
    fld = T.ConductivityField(n, 3, K, "voigt", np.full(np.prod(n), 1.0))
    r = T.solve(fld, [0.3, -0.2, 0.1], T.reference_conductivity(K), 1e-12, 10)
    assert r["iters"] == 0 and r["err"] < 1e-14  # FFT rounding only
    assert np.allclose(r["flux_mean"], K[1] * np.array([0.3, -0.2, 0.1]))


def test_fixed_point_equals_dense_solve():
    # the gradient fields satisfying div(k~ g) = 0 with mean G, written as the
    # dense linear system g + Gamma0 (k~ - k0) g = G over all voxels
    n = (5, 3, 3)
    rng = np.random.default_rng(7)
    frac = rng.random(int(np.prod(n)))
    frac[frac < 0.3] = 0.0
    fld = T.ConductivityField(n, 3, K, "voigt", frac)
    k0 = T.reference_conductivity(K)
    xi = solver.frequency_grid(n)
    m = int(np.prod(n)) * 3

    def op(v):
        g = v.reshape(n[2], n[1], n[0], 3)
        tau = fld.apply(g) - k0 * g
        out = T._gamma(np.fft.fftn(tau, axes=(0, 1, 2)), xi, k0)
        return (g - np.real(np.fft.ifftn(out, axes=(0, 1, 2)))).reshape(-1)

    A = np.stack([op(e) for e in np.eye(m)], axis=1)
    G = np.array([0.4, 0.1, -0.3])
    g_direct = np.linalg.solve(A, np.broadcast_to(G, (int(np.prod(n)), 3)).reshape(-1))
    r = T.solve(fld, G, k0, 1e-13, 20000)
    # the solve returns the update from the reported iterate: compare with that
    assert np.allclose(r["grad"].reshape(-1), g_direct, atol=1e-11)


@pytest.mark.parametrize("rule", ["voigt", "reuss", "laminate"])
def test_2d_conduction_is_antiplane_shear(rule):
    # In a 2D cell, antiplane shear (u_3(x1, x2)) of isotropic phases obeys
    # div(mu grad u_3) = 0: conduction with k = mu.  The elastic 2-layer
    # tensor has shear modulus <mu> along the layers and <1/mu>^-1 across,
    # the conduction laminate rule; Voigt and Reuss act on mu the same way.
    w = small_sphere_case(n=(15, 15, 1), dim=2, fraction=0.25, contrast=8.0, rule=rule, radius_vox=1.0,
                          subsamples=8)
    ff = F.filter_field(w)
    nrm = F.interface_normals(w.n, 2, w.spheres, ff["incl"], F.all_voxels(w.n)) if rule == "laminate" else None
    phases = (lame(1.0, 0.3), lame(8.0, 0.3))
    k = (phases[0][1], phases[1][1])
    tf = T.ConductivityField(w.n, 2, k, rule, ff["frac"], nrm)
    Kt, _ = T.effective_conductivity(tf, T.reference_conductivity(k), 1e-11, 20000, 2)
    ef = solver.StiffnessField(w.n, 2, phases, rule, ff["frac"], nrm)
    c0 = solver.reference_medium(phases)
    for j in range(2):
        E = np.zeros((3, 3))
        E[j, 2] = E[2, j] = 0.5  # gamma_j3 = 1
        r = solver.solve(ef, E, c0, 1e-11, 20000)
        s = r["sig_mean"]
        assert abs(s[0, 2] - Kt[0, j]) < 1e-7 * Kt[j, j] and abs(s[1, 2] - Kt[1, j]) < 1e-7 * Kt[j, j]
        assert np.max(np.abs(s[:2, :2])) < 1e-9 * Kt[j, j]  # no in-plane coupling
