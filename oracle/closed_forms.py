"""Exact continuum results for a slit pore with adsorption/desorption.

TEST INFRASTRUCTURE ONLY: used to pin the oracle against what the paper
states (Sec. III).

* ``adsorbed_fraction``  — Eq. 14, f_a = (1 + k_d L / (2 k_a))^-1.
* ``d_normal``           — Eq. 13, D(t) normal to the walls by inverse Laplace
  transform. As printed, the left-hand side reads D(t)/D_b while the
  right-hand side has the units of a diffusion coefficient (its t -> 0 limit
  is D_b (1 - f_a)); it is read here as D(t).
* ``taylor_aris_k``      — Eq. 15, dispersion along a Poiseuille flow. The
  leading "1" of the printed formula is read as 1/(1+2y): by Eq. 4 the
  Pe -> 0 limit of K is the long-time diffusion of the sorbing tracer along
  the walls, D_b times its mobile fraction 1/(1+2y); the Pe^2 bracket is kept
  as printed.
"""
from __future__ import annotations

import mpmath as mp


def adsorbed_fraction(k_a: float, k_d: float, L: float) -> float:
    """Eq. 14: equilibrium fraction of adsorbed tracers in a slit of width L."""
    return 1.0 / (1.0 + k_d * L / (2.0 * k_a))


def d_normal(t, k_a: float, k_d: float, L: float, d_b: float, dps: int = 40):
    """Eq. 13: time-dependent diffusion coefficient normal to the walls.

    ``t`` may be a scalar or a sequence (t > 0). Evaluated by Talbot's
    numerical inverse Laplace transform at ``dps`` decimal digits.
    """
    scalar = not hasattr(t, "__len__")
    ts = [t] if scalar else list(t)
    out = []
    with mp.workdps(dps):
        ka, kd, Lm, db = mp.mpf(k_a), mp.mpf(k_d), mp.mpf(L), mp.mpf(d_b)
        pref = 1 / (2 * ka + kd * Lm)

        def F(s):
            chi = mp.sqrt(s / db)
            kap = chi * Lm / 2
            sh, ch = mp.sinh(kap), mp.cosh(kap)
            term2 = 2 * kd * (kd + s) * sh / (chi ** 3 * ((kd + s) * ch + ka * chi * sh))
            return pref * (kd * Lm / chi ** 2 - term2)

        for tt in ts:
            out.append(float(mp.invertlaplace(F, mp.mpf(float(tt)), method="talbot")))
    return out[0] if scalar else out


def taylor_aris_k(peclet: float, k_a: float, k_d: float, L: float, d_b: float) -> float:
    """Eq. 15 (reading above): K/D_b along the flow, Pe = L vbar / D_b, y = k_a/(k_d L)."""
    y = k_a / (k_d * L)
    q = (1.0 + 2.0 * y) ** 3
    bracket = (102.0 * y * y + 18.0 * y + 1.0) / (210.0 * q) + d_b / (L * L * k_d) * 2.0 * y / q
    return 1.0 / (1.0 + 2.0 * y) + peclet * peclet * bracket


def long_time_slope(k_a: float, k_d: float, L: float, d_b: float) -> float:
    """Slope claimed in Sec. III for the intermediate-time decay, k_d/(1 + k_a L/(2 D_b))."""
    return k_d / (1.0 + k_a * L / (2.0 * d_b))
