"""Time-dependent diffusion in the compact fcc packing of spheres (Sec. III,
Figs. 4 and 5 of the paper).

One periodic unit cell of lattice parameter a (100 in the paper) holds
touching spheres of radius R = a / (2 sqrt 2) at the corners and face centres
(continuum porosity 1 - pi / (3 sqrt 2), about 26 %). The tracer diffuses at
rest (no flow) with a given fraction f_a of adsorbed tracers at equilibrium
(Eq. 14's definition: adsorbed share of the total): for a chosen k_d the
adsorption rate follows from the Eq. 11 weights,
    f_a = N_I (k_a / k_d) / (N_F + N_I k_a / k_d),
    k_a = k_d (f_a / (1 - f_a)) (N_F / N_I).
D(t) is reported against the reduced time D_b t / R^2; the medium is cubic,
so D is the mean of the three directions.

Every step runs in liblbmp's kernels; this module only draws the geometry,
solves for k_a and calls the library.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs

A_PAPER = 100
F_A_PAPER = (0.0, 0.30, 0.79, 0.97)  # Fig. 5 caption


def radius(a: int) -> float:
    return a / (2.0 * math.sqrt(2.0))


def adsorption_rates(f_a, n_fluid: int, n_iface: int, k_d: float) -> np.ndarray:
    """k_a giving the equilibrium adsorbed fraction f_a (Eq. 11 weights)."""
    f = np.asarray(f_a, dtype=np.float64)
    if np.any(f < 0) or np.any(f >= 1):
        raise ValueError("f_a must lie in [0, 1)")
    return k_d * (f / (1.0 - f)) * (n_fluid / n_iface)


def run(lb, a: int = A_PAPER, f_a=F_A_PAPER, k_d: float = 1e-3, d_b: float = 1e-2,
        t_reduced_max: float = 1.0, precision: int = 32) -> dict:
    """D(t)/D_b for each f_a, t = 0 .. t_reduced_max R^2 / D_b steps.

    Returns times (steps), t_reduced, D (n_fa, 3, T+1) in units of D_b, the
    fluid and interfacial node counts, the k_a used and the adsorbed
    fraction the run ends with."""
    mask = inputs.fcc_mask(a)
    flow = lb.lb_flow_from_velocity(mask, np.zeros((3,) + mask.shape))
    _, nf, ni = flow.classes()
    k_a = adsorption_rates(f_a, nf, ni, k_d)
    R = radius(a)
    tmax = int(math.ceil(t_reduced_max * R * R / d_b))
    mp = lb.mp_init(flow, {"D_b": d_b, "k_a": k_a, "k_d": np.full(len(k_a), k_d)}, precision, tmax)
    lb.mp_step_n(mp, tmax)
    out = lb.mp_vacf(mp, 0, 0, tmax + 1)
    mp.free()
    flow.free()
    t = np.arange(tmax + 1)
    return {"times": t, "t_reduced": d_b * t / (R * R), "D": out["D"] / d_b, "n_fluid": nf,
            "n_iface": ni, "k_a": k_a, "k_d": k_d, "d_b": d_b, "radius": R,
            "adsorbed_fraction": out["mass"][:, 1] / out["mass"].sum(axis=1)}


def main(argv=None):
    """Fig. 5: D(t)/D_b at log-spaced reduced times for the paper's f_a values;
    one JSON line."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--a", type=int, default=A_PAPER)
    ap.add_argument("--k-d", type=float, default=1e-3)
    ap.add_argument("--d-b", type=float, default=1e-2)
    ap.add_argument("--t-reduced-max", type=float, default=1.0)
    args = ap.parse_args(argv)
    from . import lbmp
    lbmp.load_library()
    r = run(lbmp, args.a, F_A_PAPER, args.k_d, args.d_b, args.t_reduced_max)
    tr = r["t_reduced"]
    idx = np.unique(np.round(np.logspace(0, math.log10(len(tr) - 1), 40)).astype(int))
    idx = np.concatenate([[0], idx])
    D = r["D"].mean(axis=1)
    print(json.dumps({"f_a": list(F_A_PAPER), "k_a": r["k_a"].tolist(), "k_d": r["k_d"], "d_b": r["d_b"],
                      "a": args.a, "radius": r["radius"], "n_fluid": r["n_fluid"], "n_iface": r["n_iface"],
                      "t_reduced": tr[idx].tolist(), "D_over_Db": D[:, idx].tolist(),
                      "adsorbed_fraction": r["adsorbed_fraction"].tolist()}))


if __name__ == "__main__":
    main()
