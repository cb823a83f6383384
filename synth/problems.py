"""Problem definitions for the five workloads and their reduced-size variants.

Parameter defaults follow the paper: the pressure-penalty prefactor tau from
Table 1 (optimal tau), velocity penalties from the appendix on penalty
parameters (boundary 10 p mu / h, intraphase 0 on Cartesian grids,
interphase C p min(mu) / h with C = 3), tau_0 = 0.5 p for the unsteady
pressure penalty of eq. (taugeneral), and V(3,3) cycles.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

from .fields import (ConstField, SinProductField, PhaseField, LogNormalRFF,
                     FourierForcing, CirclePhaseField, BubbleForcing,
                     make_exact_c1, make_exact_paper)

# Table 1 of the paper: optimal tau by (form, d), indexed by p-1.
TAU_OPTIMAL = {
    ("standard", 2): (0.19, 0.10, 0.086, 0.019, 0.031),
    ("standard", 3): (0.12, 0.088, 0.084),
    ("viscous", 2): (0.14, 0.046, 0.034, 0.0095, 0.011),
    ("viscous", 3): (0.12, 0.039, 0.040),
}


def tau_table(gamma: int, dim: int, p: int) -> float:
    form = "viscous" if gamma else "standard"
    return TAU_OPTIMAL[(form, dim)][p - 1]


@dataclass
class Problem:
    name: str
    dim: int
    n: int                          # elements per axis on the finest grid (power of two)
    p: int                          # tensor-product degree
    gamma: int                      # 0 standard form, 1 viscous-stress form
    bc: tuple                       # per axis: "periodic", "dirichlet" or "stress" (both sides)
    mu: object = field(default_factory=ConstField)
    rho: Optional[object] = None    # density field (unsteady only)
    delta: Optional[float] = None   # time-step parameter; None = steady
    phases: Optional[PhaseField] = None
    tau: Optional[float] = None
    tau0: Optional[float] = None
    tau_u_bdry_C: float = 10.0
    tau_u_inter_C: float = 3.0
    tau_u_intra_C: float = 0.0      # tau_u,0 = C p mu / h on intraphase faces
    q_cut: int = 8                  # Gauss points per piece in cut-cell quadrature
    nu1: int = 3
    nu2: int = 3
    coarsest_n: Optional[int] = None
    coloring: str = "auto"
    diag_scaling: bool = False
    exact: Optional[object] = None
    forcing: Optional[object] = None

    def __post_init__(self):
        if "stress" in self.bc and any(b != "stress" for b in self.bc):
            raise ValueError("stress boundary conditions are supported on every wall at once")
        if self.tau is None:
            self.tau = tau_table(self.gamma, self.dim, self.p)
        if self.tau0 is None:
            self.tau0 = 0.5 * self.p
        if self.coarsest_n is None:
            self.coarsest_n = 4 if self.dim == 2 else 2
        if self.coloring == "auto":
            self.coloring = default_coloring(self)

    @property
    def implicit(self) -> bool:
        """True on an implicitly defined mesh (a curved interface cuts cells)."""
        return getattr(self.phases, "kind", None) == "circle"

    @property
    def nb(self) -> int:
        return (self.dim + 1) * (self.p + 1) ** self.dim

    @property
    def n_elements(self) -> int:
        return self.n ** self.dim

    @property
    def n_dof(self) -> int:
        return self.nb * self.n_elements

    @property
    def unsteady(self) -> bool:
        return self.delta is not None and self.delta > 0

    @property
    def q_op(self) -> int:
        return self.p + 2

    @property
    def q_rhs(self) -> int:
        return self.p + 3

    @property
    def q_err(self) -> int:
        return self.p + 5

    def rhs_source(self):
        """Object providing forcing(x, chi) and forcing_div(x, chi)."""
        return self.exact if self.exact is not None else self.forcing

    def levels(self):
        """Elements per axis on each level, finest first, ending at the bottom."""
        out, n = [], self.n
        while n > self.coarsest_n:
            out.append(n)
            n //= 2
        out.append(n)
        return out


def kernel_dimension(prob: Problem) -> int:
    """Dimension of the trivial kernel (paper's footnote on the bottom solver).

    Periodic steady: constant velocity components and constant pressure;
    stress walls, steady: constant velocity components and, in viscous-stress
    form, the rigid rotations (x_a e_b - x_b e_a), pressure excluded (the
    walls fix it); unsteady with stress walls: none; otherwise (Dirichlet
    walls, or rho/delta > 0) only constant pressure.
    """
    d = prob.dim
    if all(b == "stress" for b in prob.bc):
        if prob.unsteady:
            return 0
        return d + (d * (d - 1) // 2 if prob.gamma else 0)
    periodic = all(b == "periodic" for b in prob.bc)
    if periodic and not prob.unsteady:
        return d + 1
    return 1


def default_coloring(prob: Problem) -> str:
    """Red-black for the standard form, 2^d parity for viscous-stress,
    mod-3 when interphase lifting can couple elements two apart."""
    if prob.phases is not None and prob.gamma:
        return "mod3"
    if prob.phases is not None:
        return "mod3"
    return "rb" if prob.gamma == 0 else "parity"


# ---------------------------------------------------------------------------
# The five workloads (n and p can be reduced for oracle-sized tests)
# ---------------------------------------------------------------------------
def c1_periodic_standard(n=16, p=2, nu=(2, 2)):
    """2D periodic standard-form Stokes, mu = 1, closed-form solution."""
    return Problem(name=f"c1_periodic_std_n{n}_p{p}", dim=2, n=n, p=p, gamma=0,
                   bc=("periodic", "periodic"), mu=ConstField(1.0),
                   nu1=nu[0], nu2=nu[1], coloring="rb", exact=make_exact_c1())


def c2_dirichlet_varmu(n=256, p=3, nu=(3, 3)):
    """2D viscous-stress Stokes, Dirichlet walls, mu = 1 + 0.9 sin2pi x sin2pi y."""
    mu = SinProductField(1.0, 0.9, 1.0)
    return Problem(name=f"c2_dirichlet_varmu_n{n}_p{p}", dim=2, n=n, p=p, gamma=1,
                   bc=("dirichlet", "dirichlet"), mu=mu, nu1=nu[0], nu2=nu[1],
                   coloring="parity", exact=make_exact_paper(2, 1, mu))


def c3_unsteady_periodic(n=64, p=2, re_eff=10.0, seed=0, h_ref=None):
    """3D unsteady viscous-stress Stokes, periodic, rho = mu = 1.

    delta = h^2 / Re_eff with h the finest element width (h_ref overrides it so
    that reduced grids keep the workload's delta)."""
    h = h_ref if h_ref is not None else 1.0 / n
    return Problem(name=f"c3_unsteady_n{n}_p{p}_re{re_eff:g}_s{seed}", dim=3, n=n, p=p,
                   gamma=1, bc=("periodic",) * 3, mu=ConstField(1.0), rho=ConstField(1.0),
                   delta=h * h / re_eff, coloring="parity",
                   forcing=FourierForcing.from_seed(seed, 3))


def c4a_square_inclusion(n=512, p=2, mu_in=1.0e4, mu_out=1.0):
    """2D two-phase viscous-stress Stokes: inclusion (1/4,3/4)^2, Dirichlet walls."""
    ph = PhaseField(values=(mu_in, mu_out))
    exact = make_exact_paper(2, 1, ph, phases=(1, 2), mu_chi={1: mu_in, 2: mu_out})
    return Problem(name=f"c4a_square_n{n}_p{p}", dim=2, n=n, p=p, gamma=1,
                   bc=("dirichlet", "dirichlet"), mu=ph, phases=ph, coloring="mod3",
                   diag_scaling=True, exact=exact)


def c5_lognormal(n=128, p=2, seed=1001, diag_scaling=False):
    """3D viscous-stress Stokes, Dirichlet walls, log-normal random viscosity.
    The (alpha, beta) scaling of the multi-phase section is off by default:
    for this smooth field it slows the V-cycle down (GMRES rate 0.6 without,
    0.9 with it at n = 32)."""
    mu = LogNormalRFF.from_seed(seed, 3)
    return Problem(name=f"c5_lognormal_n{n}_p{p}_s{seed}", dim=3, n=n, p=p, gamma=1,
                   bc=("dirichlet",) * 3, mu=mu, coloring="parity", diag_scaling=diag_scaling,
                   exact=make_exact_paper(3, 1, mu))


def stress_walls(dim=2, n=16, p=2, mu=None):
    """Viscous-stress Stokes with stress boundary conditions on every wall
    (sections 5.3 and 5.4): mu = 1 (section 5.3) or a given field such as
    eq. (mu); the paper's manufactured solution, h = sigma n on the walls."""
    mu = mu or ConstField(1.0)
    return Problem(name=f"stress_d{dim}_n{n}_p{p}", dim=dim, n=n, p=p, gamma=1, bc=("stress",) * dim, mu=mu,
                   coloring="parity", exact=make_exact_paper(dim, 1, mu))


def c4_circle(n=512, p=2, mu_in=1.0e4, mu_out=1.0, rhs="bubble", radius=0.3, q_cut=8):
    """2D two-phase viscous-stress Stokes on an implicitly defined mesh: a
    circle of radius 0.3 centred in the unit square cuts the n x n grid,
    viscosity mu_in inside / mu_out outside, Dirichlet walls; cut pieces below
    a quarter of a cell merged into neighbours; interphase penalty C = 8 and
    intraphase 0.5 p mu / h (appendix A for implicitly defined meshes);
    (alpha, beta) scaling.  rhs "bubble": gravity with densities 1 / 1e-3 and
    the unit surface-tension stress jump (no exact solution); rhs "exact":
    the paper's two-phase manufactured solution, its jumps as interface data."""
    ph = CirclePhaseField(values=(mu_in, mu_out), radius=radius)
    exact = forcing = None
    if rhs == "exact":
        exact = make_exact_paper(2, 1, ph, phases=(1, 2), mu_chi={1: mu_in, 2: mu_out})
    else:
        forcing = BubbleForcing(kappa=1.0 / radius)
    return Problem(name=f"c4_circle_n{n}_p{p}_{rhs}", dim=2, n=n, p=p, gamma=1,
                   bc=("dirichlet", "dirichlet"), mu=ph, phases=ph, coloring="greedy",
                   tau_u_inter_C=8.0, tau_u_intra_C=0.5, q_cut=q_cut, diag_scaling=True,
                   exact=exact, forcing=forcing)


def bubble_unsteady(n=64, p=2, water_inside=True, rhs="exact", radius=0.3):
    """The paper's multi-phase time-dependent test (section 6): a water bubble
    in gas (or a gas bubble in water) of radius 0.3 centred in the unit
    square on an implicitly defined mesh, rho 1 / 0.001 and mu 1 / 0.0002 for
    water / gas, viscous-stress form, Dirichlet walls, delta = 0.1 h (h of the
    finest grid), eq. (taugeneral) for the pressure penalty, (alpha, beta)
    scaling.  rhs "exact": the paper's two-phase manufactured solution with
    rho / delta u in its forcing and its jumps as interface data."""
    water, gas = (1.0, 1.0), (0.001, 0.0002)          # (rho, mu)
    inside, outside = (water, gas) if water_inside else (gas, water)
    mu = CirclePhaseField(values=(inside[1], outside[1]), radius=radius)
    rho = CirclePhaseField(values=(inside[0], outside[0]), radius=radius)
    delta = 0.1 / n
    exact = forcing = None
    if rhs == "exact":
        exact = make_exact_paper(2, 1, mu, phases=(1, 2), mu_chi={1: inside[1], 2: outside[1]})
        exact.rho_delta = {1: inside[0] / delta, 2: outside[0] / delta}
    else:
        forcing = BubbleForcing(rho=(inside[0], outside[0]), kappa=1.0 / radius)
    tag = "water" if water_inside else "gas"
    return Problem(name=f"bubble_{tag}_n{n}_p{p}", dim=2, n=n, p=p, gamma=1, bc=("dirichlet", "dirichlet"),
                   mu=mu, rho=rho, delta=delta, phases=mu, coloring="greedy", tau_u_inter_C=8.0,
                   tau_u_intra_C=0.5, diag_scaling=True, exact=exact, forcing=forcing)


def disk_domain(n=64, p=2, gamma=0):
    """The curved-domain test of section 5: Stokes on the unit-diameter disk
    |x - (1/2, 1/2)| < 1/2 (the domain's boundary cuts the n x n background
    grid of the unit square), mu = 1, velocity Dirichlet data on the circle
    from the paper's manufactured solution, standard form by default."""
    disk = CirclePhaseField(values=(1.0, 1.0), radius=0.5, void_outside=True)
    mu = ConstField(1.0)
    return Problem(name=f"disk_n{n}_p{p}_g{gamma}", dim=2, n=n, p=p, gamma=gamma, bc=("dirichlet", "dirichlet"),
                   mu=mu, phases=disk, coloring="greedy", tau_u_intra_C=0.5, exact=make_exact_paper(2, gamma, mu))
