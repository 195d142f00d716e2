"""Synthetic analytic EAM potential and its cubic-spline tabulation.

This module is input preparation only: it produces the tables that both the
CPU oracle and the GPU library receive as data (the paper lets rho, F and phi be
arbitrary polynomial splines, Sec. II-A, after Eq. (potential)).  Nothing here
evaluates the EAM energy or forces of a configuration.

Analytic forms (units: Angstrom, eV), the benchmark's specified potential:
    fc(r)   = (1 - (r/rc)^2)^3            for r < rc, else 0
    phi(r)  = 0.3 * exp(-8 (r/r0 - 1)) * fc(r)
    rho(r)  = exp(-6 (r/r0 - 1)) * fc(r)
    F(rho)  = -2 * sqrt(rho)
with rc = 5.0 and r0 = 2.86.  This BCC lattice at a = 3.304 is far from zero
pressure and unstable under tetragonal shear, so MD boxes collapse and heat
(hot, dense, frequent list rebuilds).

Table layout (shared convention of both consumers): a spline with n knots on
[x0, x0 + (n-1)*dx] stores, for every segment k in [0, n-2], four coefficients
c0..c3 of the cubic in the normalised local coordinate t = (x - x0)/dx - k,
t in [0, 1):  f = c0 + c1 t + c2 t^2 + c3 t^3.  Stored row-major as
coef[k, m], shape (n-1, 4), float64.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.interpolate import CubicSpline

RC = 5.0
R0 = 2.86
PHI_A = 0.3
PHI_B = 8.0
RHO_B = 6.0
EMB_A = 2.0
RHO_MAX = 40.0
N_KNOTS_MD = 2000


@dataclasses.dataclass
class SplineTable:
    """Natural cubic spline in per-segment normalised form."""

    x0: float
    dx: float
    coef: np.ndarray  # (n_knots - 1, 4) float64, c0..c3 in t

    @property
    def n_knots(self) -> int:
        return self.coef.shape[0] + 1

    @property
    def inv_dx(self) -> float:
        return 1.0 / self.dx

    @property
    def x1(self) -> float:
        return self.x0 + (self.n_knots - 1) * self.dx


SPECIFIED = dict(phi_a=PHI_A, emb_a=EMB_A)


def analytic_params(p: dict = SPECIFIED) -> dict:
    """All constants of a parameter set, for evaluators of the closed forms."""
    return dict(rc=RC, r0=R0, phi_a=p["phi_a"], phi_b=PHI_B, rho_b=RHO_B, emb_a=p["emb_a"])


# --- analytic functions (vectorised numpy) ---------------------------------

def fc(r):
    r = np.asarray(r, dtype=np.float64)
    u = 1.0 - (r / RC) ** 2
    return np.where(r < RC, u ** 3, 0.0)


def dfc(r):
    r = np.asarray(r, dtype=np.float64)
    u = 1.0 - (r / RC) ** 2
    return np.where(r < RC, 3.0 * u ** 2 * (-2.0 * r / RC ** 2), 0.0)


def _pair_core(r, p):
    r = np.asarray(r, dtype=np.float64)
    return p["phi_a"] * np.exp(-PHI_B * (r / R0 - 1.0))


def _dpair_core(r, p):
    r = np.asarray(r, dtype=np.float64)
    return p["phi_a"] * (-PHI_B / R0) * np.exp(-PHI_B * (r / R0 - 1.0))


def phi(r, p=SPECIFIED):
    return _pair_core(r, p) * fc(r)


def dphi(r, p=SPECIFIED):
    return _dpair_core(r, p) * fc(r) + _pair_core(r, p) * dfc(r)


def rho(r, p=SPECIFIED):
    return np.exp(-RHO_B * (np.asarray(r) / R0 - 1.0)) * fc(r)


def drho(r, p=SPECIFIED):
    e = np.exp(-RHO_B * (np.asarray(r) / R0 - 1.0))
    return e * (-RHO_B / R0) * fc(r) + e * dfc(r)


def emb(x, p=SPECIFIED):
    return -p["emb_a"] * np.sqrt(np.asarray(x, dtype=np.float64))


def demb(x, p=SPECIFIED):
    return -0.5 * p["emb_a"] / np.sqrt(np.asarray(x, dtype=np.float64))


def ddemb(x, p=SPECIFIED):
    return 0.25 * p["emb_a"] * np.asarray(x, dtype=np.float64) ** -1.5


# --- tabulation ---------------------------------------------------------------

def natural_spline_from_values(x0: float, dx: float, y: np.ndarray) -> SplineTable:
    """Natural cubic spline through equally spaced knot values y[k] at x0 + k dx."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    xs = x0 + dx * np.arange(n, dtype=np.float64)
    cs = CubicSpline(xs, y, bc_type="natural")
    # scipy: cs.c[m, k] multiplies (x - x_k)^(3 - m); convert to t = (x - x_k)/dx
    c = np.empty((n - 1, 4), dtype=np.float64)
    c[:, 0] = cs.c[3]
    c[:, 1] = cs.c[2] * dx
    c[:, 2] = cs.c[1] * dx ** 2
    c[:, 3] = cs.c[0] * dx ** 3
    return SplineTable(x0=float(x0), dx=float(dx), coef=c)


def tabulate(fn, x1: float, n_knots: int) -> SplineTable:
    dx = x1 / (n_knots - 1)
    xs = dx * np.arange(n_knots, dtype=np.float64)
    return natural_spline_from_values(0.0, dx, fn(xs))


def md_tables(n_knots: int = N_KNOTS_MD, rho_max: float = RHO_MAX, p: dict = SPECIFIED):
    """(phi, rho, F) tables used by every MD workload: phi, rho on [0, rc], F on [0, rho_max]."""
    return (tabulate(lambda r: phi(r, p), RC, n_knots), tabulate(lambda r: rho(r, p), RC, n_knots),
            tabulate(lambda x: emb(x, p), rho_max, n_knots))


def spline_value_map(n_knots: int) -> np.ndarray:
    """Linear map M with coef.ravel() = M @ y for a natural spline on n_knots equally spaced values.

    Built column by column from unit knot vectors (the spline is linear in y);
    independent of x0 and dx because coefficients are in the normalised t.
    """
    m = np.empty(((n_knots - 1) * 4, n_knots), dtype=np.float64)
    for k in range(n_knots):
        e = np.zeros(n_knots)
        e[k] = 1.0
        m[:, k] = natural_spline_from_values(0.0, 1.0, e).coef.ravel()
    return m


# --- force-matching model (perturbed coarse splines) --------------------------

FM_KNOTS = 64
FM_RHO_MAX = 16.0  # covers rho_i of the hottest snapshots (about 11.3)
FM_NOISE = 0.05


def fm_knot_values(seed: int = 55):
    """Knot values of the perturbed 64-knot phi, rho, F splines.

    Each analytic function is sampled at 64 equally spaced knots (phi, rho on
    [0, rc]; F on [0, 16]) and every knot value is scaled by (1 + 0.05 xi) with
    xi ~ N(0, 1) drawn from default_rng(seed) in the order phi, rho, F.
    Returns ((x1, y) for phi, rho, F).
    """
    rng = np.random.default_rng(seed)
    out = []
    for fn, x1 in ((phi, RC), (rho, RC), (emb, FM_RHO_MAX)):
        dx = x1 / (FM_KNOTS - 1)
        y = fn(dx * np.arange(FM_KNOTS))
        y = y * (1.0 + FM_NOISE * rng.standard_normal(FM_KNOTS))
        out.append((x1, y))
    return out


def fm_tables(seed: int = 55):
    tabs = []
    for x1, y in fm_knot_values(seed):
        tabs.append(natural_spline_from_values(0.0, x1 / (FM_KNOTS - 1), y))
    return tuple(tabs)


# --- a synthetic binary alloy (several atom types) -----------------------------
#
# Type 0 is the specified potential's species; type 1 is a lighter species with
# a shorter length scale and a weaker density.  Pairs (a, b) use the mean of the
# two length scales:
#     rho_t(r)   = S_t exp(-6 (r/r0_t - 1)) fc(r)
#     F_t(rho)   = -E_t sqrt(rho)
#     phi_ab(r)  = 0.3 exp(-8 (r/r0_ab - 1)) fc(r),   r0_ab = (r0_a + r0_b)/2

ALLOY_R0 = (R0, 2.72)
ALLOY_RHO_S = (1.0, 0.8)
ALLOY_EMB_A = (EMB_A, 2.4)
ALLOY_MASS = (180.95, 95.95)
# two more synthetic species of the same forms, for three- and four-type systems
# (types 0 and 1 are the binary alloy's)
MULTI_R0 = ALLOY_R0 + (2.80, 2.66)
MULTI_RHO_S = ALLOY_RHO_S + (0.9, 1.15)
MULTI_EMB_A = ALLOY_EMB_A + (2.7, 2.2)
MULTI_MASS = ALLOY_MASS + (63.55, 55.85)


def alloy_r0(a: int, b: int) -> float:
    return 0.5 * (MULTI_R0[a] + MULTI_R0[b])


def alloy_phi(r, a, b):
    return PHI_A * np.exp(-PHI_B * (np.asarray(r, dtype=np.float64) / alloy_r0(a, b) - 1.0)) * fc(r)


def alloy_dphi(r, a, b):
    r = np.asarray(r, dtype=np.float64)
    r0 = alloy_r0(a, b)
    e = PHI_A * np.exp(-PHI_B * (r / r0 - 1.0))
    return e * (-PHI_B / r0) * fc(r) + e * dfc(r)


def alloy_rho(r, t):
    r = np.asarray(r, dtype=np.float64)
    return MULTI_RHO_S[t] * np.exp(-RHO_B * (r / MULTI_R0[t] - 1.0)) * fc(r)


def alloy_drho(r, t):
    r = np.asarray(r, dtype=np.float64)
    e = MULTI_RHO_S[t] * np.exp(-RHO_B * (r / MULTI_R0[t] - 1.0))
    return e * (-RHO_B / MULTI_R0[t]) * fc(r) + e * dfc(r)


def alloy_emb(x, t):
    return -MULTI_EMB_A[t] * np.sqrt(np.asarray(x, dtype=np.float64))


def alloy_demb(x, t):
    return -0.5 * MULTI_EMB_A[t] / np.sqrt(np.asarray(x, dtype=np.float64))


def alloy_tables(n_knots: int = N_KNOTS_MD, rho_max: float = RHO_MAX, n_types: int = 2):
    """(phi[a][b], rho[t], F[t]) tables of the first n_types species (2: the
    binary alloy): phi, rho on [0, rc], F on [0, rho_max]; phi[a][b] and
    phi[b][a] are the same table."""
    nt = n_types
    assert 2 <= nt <= len(MULTI_R0)
    phi_t = [[None] * nt for _ in range(nt)]
    for a in range(nt):
        for b in range(a, nt):
            phi_t[a][b] = phi_t[b][a] = tabulate(lambda r, a=a, b=b: alloy_phi(r, a, b), RC, n_knots)
    rho_t = [tabulate(lambda r, t=t: alloy_rho(r, t), RC, n_knots) for t in range(nt)]
    emb_t = [tabulate(lambda x, t=t: alloy_emb(x, t), rho_max, n_knots) for t in range(nt)]
    return phi_t, rho_t, emb_t
