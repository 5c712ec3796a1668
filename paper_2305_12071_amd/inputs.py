"""Seeded synthetic workloads shaped like the paper's 1D argon tests.

This module only *describes* inputs: gas constants, initial/boundary states,
mesh, time step and particle weight for each case.  It contains none of the
DUWP step arithmetic (no moments, no random streams, no collision or flux
code) and imports nothing else from this package, so both the HIP path and
the oracle can be driven from it without sharing any method code.

Cases follow the paper's test section (shock structure, Sec. 4.1; Sod tube,
Sec. 4.2 and Table 1) with argon VHS constants.  The shock's downstream state
comes from the textbook Rankine-Hugoniot relations for gamma = 5/3; the mean
free path used to size a shock domain is the hard-sphere form of the paper's
Appendix A, lambda = 1 / (sqrt(2) pi d_ref^2 n).
"""
from __future__ import annotations

import json
import math
import random
from dataclasses import asdict, dataclass, field

KB = 1.380649e-23          # Boltzmann constant, J/K
GAMMA = 5.0 / 3.0          # monatomic gas

# Argon, variable-hard-sphere constants (omega = 0.81 for every case here).
AR_MASS = 6.63e-26         # kg
AR_DREF = 4.17e-10         # m
AR_OMEGA = 0.81
AR_TREF = 273.0            # K

BC_RESERVOIR = 0
BC_SPECULAR = 1

KIND_SHOCK = 0
KIND_SOD = 1
KIND_BOX = 2

CLASSIFY_RATIONAL = 0      # P = max(0, 1 - tau/dt)   (paper Eq. p)
CLASSIFY_EXP = 1           # P = 1 - exp(-dt/tau)     (QMC law, Sec. 3.2)

EPS1 = 0                   # eps_1 of Eq. vp1 (default)
EPS12 = 1                  # eps_12 = dt/(2 tau + dt)
EPS0 = 2                   # eps_0 = 1
EPS_FULL = 3               # eps of Eq. vp (time-averaged flux)


@dataclass
class Case:
    """One independent 1D case.  Units are SI for shocks, nondimensional for Sod."""
    kind: int
    ncells: int
    x_lo: float
    x_hi: float
    x_split: float
    rho_L: float
    u_L: float
    T_L: float
    rho_R: float
    u_R: float
    T_R: float
    R: float                 # specific gas constant k/m (1 for nondimensional)
    omega: float
    T_ref: float
    m_mol: float = 0.0       # molecular mass (dimensional gas) ...
    d_ref: float = 0.0       # ... and VHS reference diameter
    lambda_ref: float = 0.0  # or: reference mean free path (nondimensional gas)
    rho_ref: float = 0.0     #     at reference density rho_ref
    m_particle: float = 0.0
    dt: float = 0.0
    bc_lo: int = BC_RESERVOIR
    bc_hi: int = BC_RESERVOIR
    classify_law: int = CLASSIFY_RATIONAL
    eps_law: int = EPS1
    dsmc_full_dt: int = 0    # 1: DSMC collides over the full dt instead of (1-P) dt
    flux_order: int = 1      # 2: MUSCL-minmod inviscid face states in the wave flux
    absorb_stream: int = 0   # 1: absorbed particles stream for their free time first
    capacity: int = 0        # particle capacity hint (0 = derive)
    name: str = ""

    def to_dict(self) -> dict:
        return asdict(self)

    @property
    def dx(self) -> float:
        return (self.x_hi - self.x_lo) / self.ncells

    def domain_mass(self) -> float:
        """Initial mass per unit area (step profile at x_split)."""
        return (self.rho_L * (self.x_split - self.x_lo)
                + self.rho_R * (self.x_hi - self.x_split))


# ---------------------------------------------------------------------------
# Textbook gas dynamics used to *set up* inputs
# ---------------------------------------------------------------------------

def rankine_hugoniot(mach: float, gamma: float = GAMMA):
    """Downstream/upstream ratios (rho2/rho1, p2/p1, T2/T1, u2/u1) of a normal shock."""
    m2 = mach * mach
    r = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p = 1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0)
    return r, p, p / r, 1.0 / r


def hs_mean_free_path(n: float, d_ref: float = AR_DREF) -> float:
    """lambda = 1/(sqrt(2) pi d^2 n) (paper Appendix A)."""
    return 1.0 / (math.sqrt(2.0) * math.pi * d_ref * d_ref * n)


def vhs_beta(omega: float, alpha: float = 1.0) -> float:
    """beta of the paper's mean-free-path definition (Sec. 4.1, Eq. lambda)."""
    return 5.0 * (alpha + 1.0) * (alpha + 2.0) / (4.0 * alpha * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega))


def cfl_dt(case: Case, cfl: float = 0.3) -> float:
    """One global dt per case: cfl * dx / max over the IC states of (|u| + 4 sqrt(RT))."""
    s = max(abs(case.u_L) + 4.0 * math.sqrt(case.R * case.T_L),
            abs(case.u_R) + 4.0 * math.sqrt(case.R * case.T_R))
    return cfl * case.dx / s


# ---------------------------------------------------------------------------
# Case builders
# ---------------------------------------------------------------------------

def argon_shock(mach: float, ncells: int, length_mfp: float, n_particles: float,
                n_up: float = 1e20, T_up: float = 273.0, name: str = "") -> Case:
    """Stationary normal shock in argon; upstream enters from the left reservoir."""
    R = KB / AR_MASS
    rho1 = n_up * AR_MASS
    lam = hs_mean_free_path(n_up)
    L = length_mfp * lam
    u1 = mach * math.sqrt(GAMMA * R * T_up)
    r, _, t, _ = rankine_hugoniot(mach)
    c = Case(kind=KIND_SHOCK, ncells=ncells, x_lo=0.0, x_hi=L, x_split=0.5 * L,
             rho_L=rho1, u_L=u1, T_L=T_up, rho_R=rho1 * r, u_R=u1 / r, T_R=T_up * t,
             R=R, omega=AR_OMEGA, T_ref=AR_TREF, m_mol=AR_MASS, d_ref=AR_DREF,
             bc_lo=BC_RESERVOIR, bc_hi=BC_RESERVOIR, name=name or f"shock_M{mach:g}")
    c.dt = cfl_dt(c)
    c.m_particle = c.domain_mass() / n_particles
    return c


def sod_tube(kn: float, ncells: int, m_particle: float | None = None, dt: float | None = None,
             ppc_left: float | None = None, name: str = "") -> Case:
    """Sod tube of Table 1 (left 1,0,1; right 0.125,0,0.8), nondimensional, specular walls.

    kn is the left-state mean free path over the tube length (1).
    """
    c = Case(kind=KIND_SOD, ncells=ncells, x_lo=0.0, x_hi=1.0, x_split=0.5,
             rho_L=1.0, u_L=0.0, T_L=1.0, rho_R=0.125, u_R=0.0, T_R=0.8,
             R=1.0, omega=AR_OMEGA, T_ref=1.0, lambda_ref=kn, rho_ref=1.0,
             bc_lo=BC_SPECULAR, bc_hi=BC_SPECULAR, name=name or f"sod_Kn{kn:g}")
    c.dt = dt if dt is not None else cfl_dt(c)
    if m_particle is None:
        ppc_left = 2000.0 if ppc_left is None else ppc_left
        m_particle = c.rho_L * c.dx / ppc_left
    c.m_particle = m_particle
    return c


def box(ncells: int, rho: float, T: float, ppc: float, dt_over_tau: float,
        u: float = 0.0, cfl: float = 0.3, name: str = "") -> Case:
    """Uniform gas between specular walls.

    dt comes from the CFL rule; the reference mean free path (Kn) is then set so
    that dt/tau at the box state equals dt_over_tau, which fixes the absorbed
    fraction P.  tau = mu/p with mu = mu_ref (T/T_ref)^omega and
    mu_ref = beta Kn sqrt(2 pi) at rho_ref = R = T_ref = 1.
    """
    c = Case(kind=KIND_BOX, ncells=ncells, x_lo=0.0, x_hi=1.0, x_split=0.5,
             rho_L=rho, u_L=u, T_L=T, rho_R=rho, u_R=u, T_R=T,
             R=1.0, omega=AR_OMEGA, T_ref=1.0, lambda_ref=1.0, rho_ref=1.0,
             bc_lo=BC_SPECULAR, bc_hi=BC_SPECULAR, name=name or "box")
    c.dt = cfl_dt(c, cfl)
    tau = c.dt / dt_over_tau
    c.lambda_ref = tau * rho * T ** (1.0 - AR_OMEGA) / (vhs_beta(AR_OMEGA) * math.sqrt(2.0 * math.pi))
    c.m_particle = rho * c.dx / ppc
    return c


# Named workloads --------------------------------------------------------------

def mach3_small() -> Case:
    """Mach-3 argon shock, 100 cells over 50 upstream mean free paths, ~2e4 particles."""
    return argon_shock(3.0, 100, 50.0, 2e4, name="mach3_c100")


def sod_kn_sweep(ncells: int = 1000, n_particles: float = 1e6, dt: float = 7.5e-5):
    """Sod tubes with Kn in {1e-4 .. 1}, 1000 cells, ~1e6 particles each."""
    out = []
    for kn in (1e-4, 1e-3, 1e-2, 1e-1, 1.0):
        c = sod_tube(kn, ncells, m_particle=0.5625 / n_particles, dt=dt)
        out.append(c)
    return out


def sod_paper(kn: float) -> Case:
    """The paper's own Sod resolution: 100 cells, m_p = rho_up dx / 2000."""
    return sod_tube(kn, 100, dt=5e-4, ppc_left=2000.0, name=f"sodp_Kn{kn:g}")


def mach8_shock(ncells: int = 4000, n_particles: float = 5e7) -> Case:
    """Mach-8 argon shock, 4000 cells over 200 upstream mean free paths, 5e7 particles."""
    return argon_shock(8.0, ncells, 200.0 * ncells / 4000.0, n_particles,
                       name=f"mach8_c{ncells}")


def mach10_large(ncells: int = 20000, n_kept: float = 1e9, cell_kn: float = 1e-3,
                 kept_fraction: float = 0.028) -> Case:
    """Mach-10 argon shock in the near-continuum regime, most of the mass in the wave part.

    Cells are 1/cell_kn upstream mean free paths wide (the cell-Knudsen reading of
    "Kn = 1e-3"): 20000 cells over 2e7 mean free paths.  The particle weight puts
    about n_kept particles in the domain when they carry the fraction kept_fraction
    of the mass; 0.028 is the mass-weighted share that the absorbed fraction of the
    paper's Eq. p leaves to particles at the two reservoir states of this case
    (about 0.09 upstream and 0.012 downstream).
    """
    c = argon_shock(10.0, ncells, ncells / cell_kn, n_kept, name=f"mach10_c{ncells}")
    c.m_particle = kept_fraction * c.domain_mass() / n_kept
    c.capacity = int(1.6 * n_kept) + 4096
    return c


def batched_cases(n: int = 256, seed: int = 2305, ppc_scale: float = 1.0):
    """Independent uneven cases: half shocks (Mach ~ U[1.2,10]), half Sod (Kn log-U[1e-4,1]).

    Cells ~ U{200..2000}; particles per cell at the reference (left) state ~ U[50,500].
    """
    rng = random.Random(seed)
    out = []
    for i in range(n):
        ncells = rng.randint(200, 2000)
        ppc = rng.uniform(50.0, 500.0) * ppc_scale
        if i % 2 == 0:
            mach = rng.uniform(1.2, 10.0)
            c = argon_shock(mach, ncells, ncells / 2.0, 1.0, name=f"b{i}_shock_M{mach:.3f}")
            c.m_particle = c.rho_L * c.dx / ppc
        else:
            kn = 10.0 ** rng.uniform(-4.0, 0.0)
            c = sod_tube(kn, ncells, ppc_left=ppc, name=f"b{i}_sod_Kn{kn:.3e}")
        out.append(c)
    return out


def expected_particles(c: Case) -> float:
    return c.domain_mass() / c.m_particle


def save_manifest(cases, path: str) -> None:
    with open(path, "w") as f:
        json.dump([c.to_dict() for c in cases], f, indent=1)


def load_manifest(path: str):
    with open(path) as f:
        return [Case(**d) for d in json.load(f)]
