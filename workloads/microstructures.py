"""Seeded inclusion microstructures of the paper's kind, scaled to 3D.

The paper's single workload is a disk centred in a unit square, both phases
isotropic with the same Poisson ratio (Section 2, numerical setup).  The
generators below produce that cell and the 3D multi-inclusion cells used to
measure the solver.  Units: lengths are in voxels, the cell is
[0, n_x) x [0, n_y) x [0, n_z) and voxel ``a`` has its centre at ``a + 0.5``.
Sphere centres are placed on a 1/16-voxel lattice so that they are exact
binary fractions (they coincide with the sub-sample half-lattice for 8 and
16 sub-samples per voxel).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

# Geometry lattice: centres are multiples of 1/CENTRE_LATTICE voxel.
CENTRE_LATTICE = 16

# Rule names, matching the C enumeration order of the library.
RULES = ("none", "voigt", "reuss", "laminate")


def lame(young: float, poisson: float) -> Tuple[float, float]:
    """Lame parameters (lambda, mu) of an isotropic phase from (E, nu)."""
    lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson))
    mu = young / (2.0 * (1.0 + poisson))
    return lam, mu


@dataclasses.dataclass
class Workload:
    """One periodic cell: grid, inclusions, phases, filter and loads.

    ``spheres`` is an (k, 4) float64 array of (cx, cy, cz, r) in voxel units.
    ``phases`` is ((lambda_matrix, mu_matrix), (lambda_incl, mu_incl)).
    ``loads`` is an (n_load, 6) array of macroscopic strains, tensor
    components in the order 11, 22, 33, 23, 13, 12 (no sqrt(2) factors).
    """

    name: str
    dim: int
    n: Tuple[int, int, int]
    spheres: np.ndarray
    phases: Tuple[Tuple[float, float], Tuple[float, float]]
    radius_vox: float
    subsamples: int
    rule: str
    loads: np.ndarray
    tol: float
    max_iter: int = 10000
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nvox(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _snap(x: np.ndarray) -> np.ndarray:
    return np.round(np.asarray(x, dtype=np.float64) * CENTRE_LATTICE) / CENTRE_LATTICE


def centred_inclusion(n: int, dim: int, fraction: float) -> np.ndarray:
    """One disk (2D) or sphere (3D) of the given area/volume fraction at the cell centre.

    With odd ``n`` the cell centre n/2 is the centre of voxel (n-1)/2.
    """
    if dim == 2:
        r = math.sqrt(fraction / math.pi) * n
        return np.array([[n / 2.0, n / 2.0, 0.5, r]])
    r = (3.0 * fraction / (4.0 * math.pi)) ** (1.0 / 3.0) * n
    return np.array([[n / 2.0, n / 2.0, n / 2.0, r]])


def _min_image(d: np.ndarray, n: np.ndarray) -> np.ndarray:
    return d - n * np.round(d / n)


def rsa_spheres(rng: np.random.Generator, n: Sequence[int], radii: Sequence[float],
                gap: float, max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition of non-overlapping periodic spheres.

    Spheres are placed largest first; two spheres are accepted when their
    periodic minimum-image centre distance is at least r_i + r_j + gap.
    Raises RuntimeError when a sphere cannot be placed.
    """
    n_arr = np.asarray(n, dtype=np.float64)
    order = np.argsort(-np.asarray(radii, dtype=np.float64), kind="stable")
    placed: List[np.ndarray] = []
    prad: List[float] = []
    for idx in order:
        r = float(radii[idx])
        for _ in range(max_tries):
            c = np.mod(_snap(rng.random(3) * n_arr), n_arr)
            ok = True
            for c2, r2 in zip(placed, prad):
                d = _min_image(c - c2, n_arr)
                if float(np.sqrt(np.dot(d, d))) < r + r2 + gap:
                    ok = False
                    break
            if ok:
                placed.append(c)
                prad.append(r)
                break
        else:
            raise RuntimeError("rsa_spheres: could not place sphere %d" % len(placed))
    out = np.zeros((len(placed), 4))
    for i, (c, r) in enumerate(zip(placed, prad)):
        out[i, :3] = c
        out[i, 3] = r
    return out


def _unit_mandel_loads(dim: int) -> np.ndarray:
    """Six (3D) or three (2D, in-plane) unit Mandel strains as tensor components."""
    s = 1.0 / math.sqrt(2.0)
    rows = [
        [1, 0, 0, 0, 0, 0],
        [0, 1, 0, 0, 0, 0],
        [0, 0, 1, 0, 0, 0],
        [0, 0, 0, s, 0, 0],
        [0, 0, 0, 0, s, 0],
        [0, 0, 0, 0, 0, s],
    ]
    a = np.array(rows, dtype=np.float64)
    if dim == 2:
        return a[[0, 1, 5]]
    return a


def workload_c1(rule: str = "none") -> Workload:
    """2D plane-strain 81x81 cell, centred disk of fraction 0.2, contrast 10.

    Shear load eps_12 = 0.01, filters of radius 1 voxel with 16x16
    sub-samples, FP64 fixed point to equilibrium error 1e-8.
    """
    n = 81
    return Workload(
        name="c1-2d-81-disk",
        dim=2,
        n=(n, n, 1),
        spheres=centred_inclusion(n, 2, 0.2),
        phases=(lame(1.0, 0.3), lame(10.0, 0.3)),
        radius_vox=1.0,
        subsamples=16,
        rule=rule,
        loads=np.array([[0, 0, 0, 0, 0, 0.01]], dtype=np.float64),
        tol=1e-8,
    )


def workload_c2(contrast: float = 100.0, n: int = 125) -> Workload:
    """3D n^3 cell (125^3 by default), centred sphere of fraction 0.25.

    Contrast E_incl/E_mat in {100, 0.01}, nu = 0.3, all six unit Mandel
    strains, 2-layer filter of radius 1 voxel with 8^3 sub-samples, tol 1e-4.
    """
    return Workload(
        name="c2-3d-%d-sphere-c%g" % (n, contrast),
        dim=3,
        n=(n, n, n),
        spheres=centred_inclusion(n, 3, 0.25),
        phases=(lame(1.0, 0.3), lame(contrast, 0.3)),
        radius_vox=1.0,
        subsamples=8,
        rule="laminate",
        loads=_unit_mandel_loads(3),
        tol=1e-4,
    )


def workload_c3(seed: int = 3, radius_vox: float = 1.0, rule: str = "laminate",
                literal_radii: bool = False, n: int = 243) -> Workload:
    """3D 243^3 cell with 40 seeded non-overlapping spheres, fraction about 0.3.

    Radii are drawn uniformly in [8, 20] voxels.  Forty such spheres fill
    only about 4% of a 243^3 cell, so unless ``literal_radii`` is set all
    radii are scaled by one common factor to reach the stated total
    fraction 0.30.  Surfaces are at least 2 voxels apart.  Inclusion E = 20,
    matrix E = 1, nu = 0.3, all six loads, tol 1e-4.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    radii = rng.uniform(8.0, 20.0, size=40)
    scale = 1.0
    if not literal_radii:
        vol = float(np.sum(4.0 / 3.0 * math.pi * radii ** 3))
        scale = (0.30 * n ** 3 / vol) ** (1.0 / 3.0)
        radii = radii * scale
    sph = rsa_spheres(rng, (n, n, n), radii, gap=2.0)
    frac = float(np.sum(4.0 / 3.0 * math.pi * sph[:, 3] ** 3)) / n ** 3
    return Workload(
        name="c3-3d-%d-40spheres-r%g-%s" % (n, radius_vox, rule),
        dim=3,
        n=(n, n, n),
        spheres=sph,
        phases=(lame(1.0, 0.3), lame(20.0, 0.3)),
        radius_vox=radius_vox,
        subsamples=8,
        rule=rule,
        loads=_unit_mandel_loads(3),
        tol=1e-4,
        meta={"radius_scale": scale, "nominal_fraction": frac, "seed": seed},
    )


C4_SIZES = (45, 63, 81, 105, 125, 135)


def workload_c4(seed: int = 4, count: int = 64) -> List[Workload]:
    """A batch of seeded cells of uneven odd sizes from {45,63,81,105,125,135}^3.

    Each cell has 5-30 equal spheres at a total fraction in [0.1, 0.35] and
    an inclusion/matrix contrast log-uniform in [0.01, 100]; 2-layer filter
    of radius 1 voxel with 8^3 sub-samples, six loads, tol 1e-4.  When random
    sequential addition cannot place all spheres the count is reduced by one
    and the radius recomputed, deterministically.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for p in range(count):
        n = int(rng.choice(C4_SIZES))
        k = int(rng.integers(5, 31))
        frac = float(rng.uniform(0.10, 0.35))
        contrast = float(10.0 ** rng.uniform(-2.0, 2.0))
        sub = np.random.Generator(np.random.PCG64([seed, p]))
        while True:
            r = (3.0 * frac * n ** 3 / (4.0 * math.pi * k)) ** (1.0 / 3.0)
            try:
                sph = rsa_spheres(sub, (n, n, n), [r] * k, gap=1.0, max_tries=4000)
                break
            except RuntimeError:
                k -= 1
        out.append(Workload(
            name="c4-p%02d-%d" % (p, n),
            dim=3,
            n=(n, n, n),
            spheres=sph,
            phases=(lame(1.0, 0.3), lame(contrast, 0.3)),
            radius_vox=1.0,
            subsamples=8,
            rule="laminate",
            loads=_unit_mandel_loads(3),
            tol=1e-4,
            meta={"fraction": frac, "contrast": contrast, "count": k},
        ))
    return out


def workload_c5(seed: int = 5, n: int = 135, count: int = 25) -> Workload:
    """3D 135^3 cell with 25 seeded equal spheres at fraction 0.25, contrast 10.

    2-layer filter of radius 1 voxel with 8^3 sub-samples; the target of the
    gradient study is a seeded +-5% perturbation of the effective tensor.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    r = (3.0 * 0.25 * n ** 3 / (4.0 * math.pi * count)) ** (1.0 / 3.0)
    sph = rsa_spheres(rng, (n, n, n), [r] * count, gap=2.0)
    return Workload(
        name="c5-3d-%d-%dspheres" % (n, count),
        dim=3,
        n=(n, n, n),
        spheres=sph,
        phases=(lame(1.0, 0.3), lame(10.0, 0.3)),
        radius_vox=1.0,
        subsamples=8,
        rule="laminate",
        loads=_unit_mandel_loads(3),
        tol=1e-4,
        meta={"seed": seed},
    )


def target_perturbation(seed: int, shape: Tuple[int, int]) -> np.ndarray:
    """Seeded uniform draws in [-1, 1] used to perturb an effective tensor by +-5%."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=shape)


def small_sphere_case(n=(9, 9, 9), dim=3, fraction=0.2, contrast=10.0, rule="laminate",
                      radius_vox=1.0, subsamples=8, offset=(0.0, 0.0, 0.0)) -> Workload:
    """A small centred (optionally shifted) inclusion cell for tests."""
    nx, ny, nz = n
    if dim == 2:
        r = math.sqrt(fraction / math.pi) * nx
        sph = np.array([[nx / 2.0 + offset[0], ny / 2.0 + offset[1], 0.5, r]])
    else:
        r = (3.0 * fraction / (4.0 * math.pi)) ** (1.0 / 3.0) * nx
        sph = np.array([[nx / 2.0 + offset[0], ny / 2.0 + offset[1], nz / 2.0 + offset[2], r]])
    return Workload(
        name="small-%dx%dx%d" % (nx, ny, nz),
        dim=dim,
        n=(nx, ny, nz),
        spheres=sph,
        phases=(lame(1.0, 0.3), lame(contrast, 0.3)),
        radius_vox=radius_vox,
        subsamples=subsamples,
        rule=rule,
        loads=_unit_mandel_loads(dim),
        tol=1e-4,
    )


def random_fraction_case(seed: int, n=(9, 7, 5)) -> np.ndarray:
    """A seeded per-voxel fraction field in [0, 1] with exact 0 and 1 entries.

    Laid out [z][y][x] (x fastest); a quarter of the voxels are pure matrix,
    a quarter pure inclusion and the rest fractional.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = n
    f = rng.random((nz, ny, nx))
    u = rng.random((nz, ny, nx))
    f[u < 0.25] = 0.0
    f[u > 0.75] = 1.0
    return f


# Resolutions of the resolution study: the odd sizes between 7 and 125 whose
# prime factors are 3, 5, 7, 11 and 13 (the paper sweeps every size from 6
# to 128).
FIG1_RESOLUTIONS = (7, 9, 11, 13, 15, 21, 25, 27, 33, 35, 39, 45, 49, 55, 63, 65, 75, 77, 81, 91, 99, 105, 117,
                    121, 125)
FIG1_DISK_RADIUS = math.pi / 15.0  # cell lengths (Section 2 numerical setup)


def fig1_disk_case(n: int, contrast: float, rule: str = "none", radius_vox: float = 0.55,
                   subsamples: int = 16) -> Workload:
    """The 2D cell of the resolution study: a disk of radius pi/15 centred in
    the unit square, n x n pixels, E_inclusion / E_matrix = contrast with
    nu = 0.3 in both phases, loaded by a uniaxial mean strain of 1 %."""
    r = FIG1_DISK_RADIUS * n
    sph = np.array([[n / 2.0, n / 2.0, 0.5, r]])
    loads = np.zeros((1, 6))
    loads[0, 0] = 0.01
    return Workload(
        name="fig1-%d-c%g-%s-r%g" % (n, contrast, rule, radius_vox),
        dim=2,
        n=(n, n, 1),
        spheres=sph,
        phases=(lame(1.0, 0.3), lame(contrast, 0.3)),
        radius_vox=radius_vox,
        subsamples=subsamples,
        rule=rule,
        loads=loads,
        tol=1e-4,
        meta={"contrast": contrast},
    )


def rotation_from_seed(seed: int) -> np.ndarray:
    """A seeded proper rotation (3x3, columns orthonormal, det +1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


_MANDEL_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def cubic_mandel(c11: float, c12: float, c44: float, R=None) -> np.ndarray:
    """Mandel 6x6 matrix of a cubic crystal (Voigt constants C11, C12, C44)
    whose cube axes are the columns of R (the identity when R is None)."""
    c = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            c[i, i, j, j] = c11 if i == j else c12
            if i != j:
                c[i, j, i, j] = c[i, j, j, i] = c44
    if R is not None:
        c = np.einsum("ai,bj,ck,dl,ijkl->abcd", R, R, R, R, c)
    w = np.array([1.0, 1.0, 1.0, math.sqrt(2.0), math.sqrt(2.0), math.sqrt(2.0)])
    m = np.zeros((6, 6))
    for A, (i, j) in enumerate(_MANDEL_PAIRS):
        for B, (k, l) in enumerate(_MANDEL_PAIRS):
            m[A, B] = w[A] * w[B] * c[i, j, k, l]
    return m


def iso_mandel(lam: float, mu: float) -> np.ndarray:
    """Mandel 6x6 matrix of an isotropic phase."""
    m = np.zeros((6, 6))
    m[:3, :3] = lam
    m += 2.0 * mu * np.eye(6)
    return m


def workload_aniso(n: int = 125, seed: int = 8) -> Workload:
    """The n^3 centred-sphere cell (fraction 0.25) with an isotropic matrix
    (E = 1, nu = 0.3) and a cubic inclusion (C11, C12, C44 = 30, 12, 20)
    whose cube axes take a seeded rotation; 2-layer filter r = 1 voxel with
    8^3 sub-samples, six unit loads, tol 1e-4.  meta["C_mandel"] holds the
    two phase Mandel matrices."""
    cm = np.stack([iso_mandel(*lame(1.0, 0.3)), cubic_mandel(30.0, 12.0, 20.0, rotation_from_seed(seed))])
    return Workload(
        name="aniso-3d-%d-cubic-sphere" % n,
        dim=3,
        n=(n, n, n),
        spheres=centred_inclusion(n, 3, 0.25),
        phases=(lame(1.0, 0.3), lame(1.0, 0.3)),
        radius_vox=1.0,
        subsamples=8,
        rule="laminate",
        loads=_unit_mandel_loads(3),
        tol=1e-4,
        meta={"C_mandel": cm, "seed": seed},
    )


def workload_nphase(seed: int = 6, n: int = 125, count: int = 20, rule: str = "voigt") -> Workload:
    """Three-phase n^3 cell: `count` seeded non-overlapping spheres (radii
    U[10, 16] voxels, surfaces 2 voxels apart) labelled alternately 1 and 2;
    phases E = 1 (matrix), 20 and 0.05, nu = 0.3; filter r = 1 voxel with
    8^3 sub-samples; six unit loads, tol 1e-4.  meta["labels"] holds the
    sphere labels and meta["phases"] the three Lame pairs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    radii = rng.uniform(10.0, 16.0, size=count)
    sph = rsa_spheres(rng, (n, n, n), radii, gap=2.0)
    labels = np.array([1 + (i % 2) for i in range(sph.shape[0])], dtype=np.int32)
    phases = [lame(1.0, 0.3), lame(20.0, 0.3), lame(0.05, 0.3)]
    return Workload(
        name="nphase-3d-%d-%dspheres" % (n, count),
        dim=3,
        n=(n, n, n),
        spheres=sph,
        phases=(phases[0], phases[1]),
        radius_vox=1.0,
        subsamples=8,
        rule=rule,
        loads=_unit_mandel_loads(3),
        tol=1e-4,
        meta={"labels": labels, "phases": phases, "seed": seed},
    )


def thin_grid_case(length: int, axis: int, seed: int = 12, contrast: float = 10.0, rule: str = "laminate",
                   radius_vox: float = 1.0, subsamples: int = 4, thin=(9, 15), fraction: float = 0.15) -> Workload:
    """A slab cell that is `length` voxels long along `axis` and thin (9 and
    15 voxels) along the other two, holding a seeded row of small
    non-overlapping spheres (radii in [2.5, 4] voxels, fraction about 0.15):
    every line length of the solver's transforms can then be put on any axis
    at a size the oracle runs in seconds."""
    n = [0, 0, 0]
    others = [a for a in range(3) if a != axis]
    n[axis] = int(length)
    n[others[0]], n[others[1]] = int(thin[0]), int(thin[1])
    rng = np.random.Generator(np.random.PCG64(seed + 1000 * axis + length))
    vol = float(n[0] * n[1] * n[2])
    radii = []
    while sum(4.0 / 3.0 * math.pi * r ** 3 for r in radii) < fraction * vol:
        radii.append(float(rng.uniform(2.5, 4.0)))
    sph = rsa_spheres(rng, n, radii, gap=1.0)
    return Workload(
        name="thin-%dx%dx%d" % tuple(n),
        dim=3,
        n=tuple(n),
        spheres=sph,
        phases=(lame(1.0, 0.3), lame(contrast, 0.3)),
        radius_vox=radius_vox,
        subsamples=subsamples,
        rule=rule,
        loads=_unit_mandel_loads(3),
        tol=1e-4,
    )
