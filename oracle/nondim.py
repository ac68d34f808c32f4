"""Nondimensional numbers and closed-form LEFM checks (oracle test
utilities).

* Plane-strain KGD toughness and viscosity numbers (Sec. "Verification of the
  fully-coupled algorithm"):  K = (12 mu Q0 E'^3)^(-1/4) (8/sqrt(2 pi)) K_IC,
  M = 12 mu Q0 E'^3 (8/sqrt(2 pi) K_IC)^-4, K_IC = sqrt(G_c E'), K = M^(-1/4).
* Radial (penny) numbers (Sec. "... penny-shaped crack"):
  K(t) = (t^2 / ((12 mu)^5 Q0^3 E'^13))^(1/18) (8/sqrt(2 pi)) K_IC,
  M(t) = 12 mu (Q0^3 E'^13 / t^2)^(1/5) (8/sqrt(2 pi) K_IC)^(-18/5),
  M = K^(-18/5).
* E' is the plane-strain modulus E / (1 - nu^2) (the paper names it without
  printing the formula; this reading reproduces its printed K and M).
* Sneddon's openings of a crack under uniform pressure p in an infinite
  medium (textbook LEFM, not printed in the paper):
  2D w(x) = (4 p / E') sqrt(l^2 - x^2), volume 2 pi p l^2 / E';
  penny w(r) = (8 p / (pi E')) sqrt(R^2 - r^2), volume 16 p R^3 / (3 E').
"""
from __future__ import annotations

import math

KC = 8.0 / math.sqrt(2.0 * math.pi)


def e_prime(E: float, nu: float) -> float:
    return E / (1.0 - nu * nu)


def k_ic(G_c: float, E: float, nu: float) -> float:
    return math.sqrt(G_c * e_prime(E, nu))


def kgd_toughness(E, nu, mu, Q0, G_c) -> float:
    Ep = e_prime(E, nu)
    return (12.0 * mu * Q0 * Ep ** 3) ** -0.25 * KC * k_ic(G_c, E, nu)


def kgd_viscosity(E, nu, mu, Q0, G_c) -> float:
    Ep = e_prime(E, nu)
    return 12.0 * mu * Q0 * Ep ** 3 * (KC * k_ic(G_c, E, nu)) ** -4


def penny_toughness(t, E, nu, mu, Q0, G_c) -> float:
    Ep = e_prime(E, nu)
    return (t * t / ((12.0 * mu) ** 5 * Q0 ** 3 * Ep ** 13)) ** (1.0 / 18.0) * KC * k_ic(G_c, E, nu)


def penny_viscosity(t, E, nu, mu, Q0, G_c) -> float:
    Ep = e_prime(E, nu)
    return 12.0 * mu * (Q0 ** 3 * Ep ** 13 / (t * t)) ** 0.2 * (KC * k_ic(G_c, E, nu)) ** (-18.0 / 5.0)


def penny_time_for_toughness(K_target, E, nu, mu, Q0, G_c) -> float:
    """Time at which the radial toughness number reaches K_target
    (K grows like t^(1/9))."""
    k1 = penny_toughness(1.0, E, nu, mu, Q0, G_c)
    return (K_target / k1) ** 9


def sneddon_opening_2d(x, p, half_length, Ep):
    return 4.0 * p / Ep * math.sqrt(max(half_length ** 2 - x * x, 0.0))


def sneddon_volume_2d(p, half_length, Ep):
    return 2.0 * math.pi * p * half_length ** 2 / Ep


def sneddon_volume_penny(p, R, Ep):
    return 16.0 * p * R ** 3 / (3.0 * Ep)


def kgd_uniform_pressure_increment(Q0, dt, half_length, Ep):
    """Pressure rise of a fixed-length plane-strain crack under uniform
    pressure when Q0 dt is injected: volume 2 pi p l^2 / E' is linear in p."""
    return Ep * Q0 * dt / (2.0 * math.pi * half_length ** 2)
