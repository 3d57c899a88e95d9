"""Time-dependent diffusion and dispersion in a random porous medium: the
256^3 periodic Boolean sphere pack (radius 8, porosity 0.4) with flow at
Pe = 10 and 16 species, D(t) sampled on a logarithmic time grid.

The flow is the BGK solution at a small reference force, rescaled to the
target Peclet number on the sample length (Stokes regime: the steady velocity
is linear in the force). Every step runs in liblbmp's kernels; this module
draws the medium and the rates, calls the library and samples the series.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs

N, RADIUS, POROSITY, N_SPECIES, SEED = 256, 8, 0.4, 16, 2024
D_B, PECLET = 1e-2, 10.0
G_REF, FLOW_TOL = 1e-6, 1e-10  # reference force of the flow solve, steady-state tolerance


def build(lb, n: int = N, radius: float = RADIUS, porosity: float = POROSITY, n_species: int = N_SPECIES,
          seed: int = SEED, d_b: float = D_B, peclet: float = PECLET, log=None):
    """(flow, species) of the medium; species (k_a, k_d) log-uniform in [1e-4, 1e-1]."""
    t0 = time.time()
    mask = inputs.sphere_pack(n, radius, porosity, seed=seed)
    if log:
        log(f"sphere pack {n}^3: {time.time() - t0:.1f}s")
    t0 = time.time()
    ref = lb.lb_flow_solve(mask, 1.0, [G_REF, 0.0, 0.0], FLOW_TOL, 400000)
    u = ref.velocity()
    ref.free()
    vbar = float(u[0][mask == 0].mean())
    u *= (peclet * d_b / n) / vbar
    flow = lb.lb_flow_from_velocity(mask, u)
    if log:
        log(f"flow: {time.time() - t0:.1f}s")
    ka, kd = inputs.loguniform_rates(n_species, 1e-4, 1e-1, seed=seed + 2)
    return flow, {"D_b": d_b, "k_a": ka, "k_d": kd}


def log_grid(tmax: int, per_decade: int = 10) -> np.ndarray:
    """t = 0 and about per_decade log-spaced integer times per decade up to tmax."""
    n = int(math.ceil(per_decade * math.log10(max(tmax, 1)))) + 1
    return np.unique(np.concatenate([[0], np.round(np.logspace(0, math.log10(tmax), n)).astype(np.int64)]))


def run(lb, steps: int, per_decade: int = 10, precision: int = 32, log=None, **kw) -> dict:
    """D(t) / D_b (species, direction, grid time) on the log grid, the mass
    totals at the end and the propagation time per step."""
    flow, species = build(lb, log=log, **kw)
    mp = lb.mp_init(flow, species, precision, steps)
    import torch
    torch.cuda.synchronize()
    t0 = time.time()
    chunk = 10000  # report progress every chunk of steps
    for done in range(0, steps, chunk):
        lb.mp_step_n(mp, min(chunk, steps - done))
        mp.stream.synchronize()
        if log:
            log(f"steps {min(done + chunk, steps)}/{steps}: {time.time() - t0:.1f}s")
    el = time.time() - t0
    out = lb.mp_vacf(mp, 0, 0, steps + 1)
    grid = log_grid(steps, per_decade)
    st = lb.mp_stats(mp, 0)
    mp.free()
    d_b = species["D_b"]
    return {"t": grid, "D": out["D"][:, :, grid] / d_b, "mass": out["mass"], "vbar": out["vbar"],
            "k_a": species["k_a"], "k_d": species["k_d"], "n_fluid": st["n_fluid"], "n_iface": st["n_iface"],
            "ms_per_step": el / steps * 1e3, "flow": flow}


def main(argv=None):
    """One JSON line: the log-grid D(t)/D_b of every species (x along the flow)."""
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--per-decade", type=int, default=10)
    args = ap.parse_args(argv)
    from . import lbmp
    lbmp.load_library()
    r = run(lbmp, args.steps, args.per_decade, n=args.n, log=lambda m: print(m, file=sys.stderr, flush=True))
    r["flow"].free()
    print(json.dumps({"n": args.n, "steps": args.steps, "t": r["t"].tolist(), "k_a": r["k_a"].tolist(),
                      "k_d": r["k_d"].tolist(), "n_fluid": r["n_fluid"], "n_iface": r["n_iface"],
                      "ms_per_step": r["ms_per_step"],
                      "mass_error_max": float(np.abs(r["mass"].sum(axis=1) - 1).max()),
                      "D_over_Db": np.round(r["D"], 6).tolist()}))


if __name__ == "__main__":
    main()
