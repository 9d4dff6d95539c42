"""Pins of the oracle's conjugate-gradient solve (the Krylov alternative of
Section 5) against properties the mathematics fixes: G is an orthogonal
projection, G c~ G is symmetric positive definite, CG residuals are mutually
orthogonal, and the CG limit is the fixed point of the basic scheme (eqs. 1-2)."""
import numpy as np

from oracle import filter as F, solver
from workloads import fig1_disk_case, small_sphere_case


def _field(n, contrast, rule="laminate"):
    w = small_sphere_case(n=(n, n, n), contrast=contrast, rule=rule, radius_vox=1.0, subsamples=4)
    ff = F.filter_field(w)
    nrm = F.interface_normals(w.n, 3, w.spheres, ff["incl"], F.all_voxels(w.n)) if rule == "laminate" else None
    return w, solver.StiffnessField(w.n, 3, w.phases, rule, ff["frac"], nrm)


def _random_sym(rng, n):
    a = rng.standard_normal((n[2], n[1], n[0], 3, 3))
    return 0.5 * (a + np.swapaxes(a, -1, -2))


def test_projection_is_orthogonal_and_kills_constants():
    rng = np.random.default_rng(3)
    n = (7, 5, 9)
    xi = solver.frequency_grid(n)
    u, v = _random_sym(rng, n), _random_sym(rng, n)
    Gu, Gv = solver.project_compatible(u, xi), solver.project_compatible(v, xi)
    assert np.allclose(solver.project_compatible(Gu, xi), Gu, atol=1e-12)  # idempotent
    assert abs(solver.field_dot(Gu, v) - solver.field_dot(u, Gv)) < 1e-10 * np.sqrt(
        solver.field_dot(u, u) * solver.field_dot(v, v))  # self-adjoint
    const = np.broadcast_to(solver.strain_tensor([1, 2, 3, 4, 5, 6]), u.shape)
    assert np.allclose(solver.project_compatible(const, xi), 0.0, atol=1e-12)
    # a symmetric gradient of a periodic displacement is compatible: G leaves it
    nx, ny, nz = n
    disp_hat = np.fft.fftn(rng.standard_normal((nz, ny, nx, 3)), axes=(0, 1, 2))
    grad = 1j * np.einsum("zyxi,zyxj->zyxij", disp_hat, xi)
    g = np.real(np.fft.ifftn(0.5 * (grad + np.swapaxes(grad, -1, -2)), axes=(0, 1, 2)))
    assert np.allclose(solver.project_compatible(g, xi), g, atol=1e-9 * np.abs(g).max())


def test_galerkin_operator_is_symmetric_positive():
    rng = np.random.default_rng(4)
    w, fld = _field(7, 30.0)
    xi = solver.frequency_grid(w.n)
    u = solver.project_compatible(_random_sym(rng, w.n), xi)
    v = solver.project_compatible(_random_sym(rng, w.n), xi)
    Au = solver.project_compatible(fld.apply(u), xi)
    Av = solver.project_compatible(fld.apply(v), xi)
    s = np.sqrt(solver.field_dot(Au, Au) * solver.field_dot(v, v))
    assert abs(solver.field_dot(Au, v) - solver.field_dot(u, Av)) < 1e-10 * s
    assert solver.field_dot(u, Au) > 0.0


def test_cg_residuals_are_orthogonal():
    w, fld = _field(7, 30.0)
    r = solver.solve_cg(fld, [0.01, 0, 0, 0, 0.002, 0], 1e-30, 8, keep_residuals=True)
    rs = r["residuals"]
    for i in range(len(rs)):
        for j in range(i):
            d = solver.field_dot(rs[i], rs[j])
            assert abs(d) < 1e-8 * np.sqrt(solver.field_dot(rs[i], rs[i]) * solver.field_dot(rs[j], rs[j]))


def test_cg_limit_is_the_basic_fixed_point_in_far_fewer_iterations():
    w, fld = _field(9, 100.0)
    c0 = solver.reference_medium(w.phases)
    for E in ([0.01, 0, 0, 0, 0, 0], [0, 0, 0, 0.004, 0, 0.01]):
        b = solver.solve(fld, E, c0, 1e-9, 20000)
        c = solver.solve_cg(fld, E, 1e-9, 2000)
        assert b["status"] == solver.STATUS_CONVERGED and c["status"] == solver.STATUS_CONVERGED
        assert np.max(np.abs(c["sig_mean"] - b["sig_mean"])) < 1e-8 * np.max(np.abs(b["sig_mean"]))
        assert c["iters"] * 4 < b["iters"]
        # the returned field is the iterate itself: mean E, stress mean as reported
        assert np.allclose(np.mean(c["eps"].reshape(-1, 3, 3), axis=0), solver.strain_tensor(E), atol=1e-14)


def test_cg_through_the_high_contrast_mean_stress_swing():
    # the 2D disk at contrast 1e3 whose basic iterates swing the mean stress
    w = fig1_disk_case(7, 1e3, "none")
    ff = F.filter_field(w)
    fld = solver.StiffnessField(w.n, 2, w.phases, "none", ff["frac"], None)
    E = [0, 0, 0, 0, 0, 0.01]
    b = solver.solve(fld, E, solver.reference_medium(w.phases), 1e-10, 20000)
    c = solver.solve_cg(fld, E, 1e-10, 2000)
    assert c["status"] == solver.STATUS_CONVERGED
    assert abs(c["sig_mean"][0, 1] - b["sig_mean"][0, 1]) < 1e-8 * abs(b["sig_mean"][0, 1])
    assert c["iters"] * 4 < b["iters"]
