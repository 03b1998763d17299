"""Plasma-parameter calculator for the relativistic double Harris sheet.

Gaussian units throughout.  The code units used by the workloads are
c = m_e = e = 1 and omega_pe0 = 1, so the sheet-centre density per species is
n0 = 1/(4 pi).

Formulas (Schoeffler et al. 2025, Sec. 2 "Methods and Simulation Setup"):
  * cold and hot magnetisation, sigma_c = B0^2/(4 pi n m c^2) and
    sigma_h = B0^2/(4 pi n h) with h ~ 4T (the two magnetisation equations of
    the introduction);
  * pressure balance B0 = sqrt(8 pi (2 n0) T / Gamma_d) (equation "forcebalance");
  * Ampere's law for the half thickness a = c B0 / (4 pi e (2 n0) v_d)
    (equation "ampere");
  * inertial lengths and Larmor radii (equations "classde", "relde",
    "classrho", "relrho", "classdeb").

This module is input preparation only: it holds none of the particle or
field-solve arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


def gamma_from_proper(u: float) -> float:
    """Lorentz factor for a proper speed u = Gamma v (units of c)."""
    return math.sqrt(1.0 + u * u)


def gamma_from_beta(beta: float) -> float:
    return 1.0 / math.sqrt(1.0 - beta * beta)


@dataclass(frozen=True)
class HarrisParams:
    """Derived parameters of one double Harris sheet (Sec. 2)."""

    n0: float          # sheet-centre density per species
    T: float           # temperature (energy units, same for all species)
    beta_d: float      # drift speed v_d / c
    Gamma_d: float     # drift Lorentz factor
    u_d: float         # proper drift speed Gamma_d v_d / c
    B0: float          # asymptotic field from pressure balance
    a: float           # sheet half thickness from Ampere's law
    c: float = 1.0
    e: float = 1.0


def harris(n0: float, T: float, beta_d: float, c: float = 1.0, e: float = 1.0) -> HarrisParams:
    """B0 from pressure balance and a from Ampere's law (Sec. 2).

    The factor 2 n0 is the total (both species) sheet-centre density.
    """
    Gd = gamma_from_beta(beta_d)
    B0 = math.sqrt(8.0 * math.pi * (2.0 * n0) * T / Gd)
    a = c * B0 / (4.0 * math.pi * e * (2.0 * n0) * beta_d * c)
    return HarrisParams(n0=n0, T=T, beta_d=beta_d, Gamma_d=Gd, u_d=Gd * beta_d, B0=B0, a=a, c=c, e=e)


def sigma_cold(B0: float, n: float, m: float, c: float = 1.0) -> float:
    """Cold magnetisation sigma_c = B0^2 / (4 pi n m c^2) (Sec. 1)."""
    return B0 * B0 / (4.0 * math.pi * n * m * c * c)


def sigma_hot(B0: float, n: float, T: float) -> float:
    """Hot magnetisation with the ultra-relativistic enthalpy h = 4T (Sec. 1)."""
    return B0 * B0 / (4.0 * math.pi * n * 4.0 * T)


def n0_over_nb_for_sigma(sigma_c: float, T: float, m: float, u_d: float, c: float = 1.0) -> float:
    """Sheet-to-background density ratio that gives a cold magnetisation sigma_c.

    Inserting pressure balance into sigma_c = B0^2/(4 pi n_b m c^2) gives
    sigma_c = 4 (n0/n_b) T / (Gamma_d m c^2) (Sec. 2, Sec. 3.2).
    """
    Gd = gamma_from_proper(u_d / c)
    return sigma_c * Gd * m * c * c / (4.0 * T)


def inertial_length_classical(m: float, n: float, c: float = 1.0, e: float = 1.0) -> float:
    """d_C = sqrt(m c^2 / (4 pi n e^2)) (equation "classde")."""
    return math.sqrt(m * c * c / (4.0 * math.pi * n * e * e))


def thermal_speed(T: float, m: float, c: float = 1.0) -> float:
    """v_T / c = sqrt(2T/(m c^2)) (Sec. 2, classical regime)."""
    return math.sqrt(2.0 * T / (m * c * c))


def larmor_classical_over_a(T: float, m: float, u_d: float, c: float = 1.0) -> float:
    """rho_{L,C} / a = u_d / v_T (equation "classrho")."""
    return u_d / (thermal_speed(T, m, c) * c)


def larmor_relativistic_over_a(u_d: float, c: float = 1.0) -> float:
    """rho_{L,R} / a = u_d / c (equation "relrho")."""
    return u_d / c


def larmor_relativistic(T: float, m: float, u_d: float, n0: float, c: float = 1.0, e: float = 1.0) -> float:
    """rho_{L,R} = sqrt(Gamma_d/2) sqrt(Gamma_T) d_{0,C} with Gamma_T = 2T/(m c^2)
    (equations "relde" and "relrho")."""
    Gd = gamma_from_proper(u_d / c)
    GT = 2.0 * T / (m * c * c)
    return math.sqrt(Gd / 2.0) * math.sqrt(GT) * inertial_length_classical(m, n0, c, e)


def nominal_larmor(B0: float, m: float, c: float = 1.0, e: float = 1.0) -> float:
    """rho_0 = c / Omega_c with Omega_c = e B0 / (m c) (Sec. 2)."""
    return m * c * c / (e * B0)
