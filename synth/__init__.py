"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This package holds problem *data* only: the grid, degree, Stokes form,
boundary conditions, coefficient fields (viscosity, density), manufactured
solutions and forcing functions, each evaluated pointwise in closed form.
It contains none of the discretisation or solver arithmetic; the oracle and
the HIP library each build their operators from these definitions in code of
their own.
"""
from .problems import (Problem, c1_periodic_standard, c2_dirichlet_varmu,
                       c3_unsteady_periodic, c4a_square_inclusion,
                       c5_lognormal, stress_walls, c4_circle, bubble_unsteady, disk_domain, TAU_OPTIMAL, kernel_dimension)
from .fields import (ConstField, SinProductField, PhaseField, LogNormalRFF,
                     FourierForcing, CirclePhaseField, BubbleForcing,
                     make_exact_c1, make_exact_paper)

__all__ = [
    "Problem", "c1_periodic_standard", "c2_dirichlet_varmu",
    "c3_unsteady_periodic", "c4a_square_inclusion", "c5_lognormal", "stress_walls",
    "TAU_OPTIMAL", "kernel_dimension", "ConstField", "SinProductField",
    "PhaseField", "LogNormalRFF", "FourierForcing", "make_exact_c1",
    "make_exact_paper", "c4_circle", "bubble_unsteady", "disk_domain", "CirclePhaseField", "BubbleForcing",
]
