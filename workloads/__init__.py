"""Seeded synthetic inputs for the filtered-property Lippmann-Schwinger solver.

This package only draws geometries (inclusion centres and radii), phase
moduli and macroscopic loads from fixed seeds.  It contains none of the
method's arithmetic (no filter, no homogenisation rule, no Green operator),
so that the oracle and the GPU path can both consume the same inputs while
sharing no computation.
"""
from .microstructures import (  # noqa: F401
    Workload,
    lame,
    centred_inclusion,
    rsa_spheres,
    workload_c1,
    workload_c2,
    workload_c3,
    workload_c4,
    workload_c5,
    small_sphere_case,
    target_perturbation,
    random_fraction_case,
    fig1_disk_case,
    FIG1_RESOLUTIONS,
    FIG1_DISK_RADIUS,
    workload_aniso,
    workload_nphase,
    thin_grid_case,
    cubic_mandel,
    iso_mandel,
    rotation_from_seed,
)
