"""Writes ``c4_sphere64_dt.json``: FP64 oracle D(t) of a 64^3 Boolean sphere
pack (radius 8, porosity 0.4, the generator of the 256^3 porous workload) with
its BGK flow at Pe = 10, for 4 species spanning K = k_a/k_d, over 2e5 steps,
sampled on a logarithmic time grid.

Calls only ``oracle`` (flow, propagation, D(t)) and ``paper_1303_2470_amd.inputs``
(the seeded sphere pack). Nothing here comes from the GPU path.

Recipe (Sec. I Eq. 6 for the flow; Sec. II Eqs. 7-12 for the tracer):
  * mask = inputs.sphere_pack(64, 8, 0.4, seed=2024);
  * steady BGK flow (tau = 1, Guo forcing, half-way bounce-back) at the
    reference force g = (1e-6, 0, 0) to a relative step change of 1e-10;
  * velocity rescaled to the mean fluid velocity Pe D_b / 64 along x (Stokes
    regime: the steady velocity is linear in the force), Pe = 10, D_b = 1e-2;
  * x and z first moments propagated for 2e5 steps per species, D(t) of the
    discrete Eq. 3 about the mean drift.

Run: ``OMP_NUM_THREADS=8 python tests/golden/make_c4_ref.py`` (a few CPU hours;
the file is rewritten after every species).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1303_2470_amd import inputs  # noqa: E402

N, RADIUS, POROSITY, SEED = 64, 8, 0.4, 2024
D_B, PECLET, G_REF, FLOW_TOL = 1e-2, 10.0, 1e-6, 1e-10
STEPS = 200_000
# (k_a, k_d): K = k_a / k_d = 1e-3, 0.2, 5, 30; exchange times 10 to 1000 steps
SPECIES = [(1e-4, 1e-1), (2e-3, 1e-2), (1e-2, 2e-3), (3e-2, 1e-3)]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_sphere64_dt.json")


def log_grid(tmax: int, per_decade: int = 10) -> np.ndarray:
    n = int(math.ceil(per_decade * math.log10(tmax))) + 1
    return np.unique(np.concatenate([[0], np.round(np.logspace(0, math.log10(tmax), n)).astype(np.int64)]))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=STEPS)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args(argv)
    t0 = time.time()
    mask = inputs.sphere_pack(N, RADIUS, POROSITY, seed=SEED)
    fl = oracle.bgk(mask, 1.0, [G_REF, 0.0, 0.0], tol=FLOW_TOL, max_steps=400_000)
    if not fl["converged"]:
        raise SystemExit("flow did not converge")
    u = fl["u"]
    fluid = mask == 0
    ux_ref = float(u[0][fluid].mean())
    u = u * ((PECLET * D_B / N) / ux_ref)
    print(f"flow: {fl['steps']} steps, residual {fl['residual']:.3e}, mean u_x {ux_ref:.12e}, "
          f"{time.time() - t0:.0f}s", flush=True)
    grid = log_grid(args.steps)
    cls = oracle.classify(mask)
    rec = {
        "_about": __doc__.strip().splitlines()[0] + " Written by tests/golden/make_c4_ref.py.",
        "n": N, "radius": RADIUS, "porosity": POROSITY, "seed": SEED,
        "D_b": D_B, "peclet": PECLET, "g_ref": G_REF, "flow_tol": FLOW_TOL,
        "flow_steps": fl["steps"], "flow_residual": fl["residual"], "mean_ux_ref": ux_ref,
        "n_fluid": int((cls > 0).sum()), "n_iface": int((cls == 2).sum()),
        "steps": args.steps, "t": grid.tolist(), "k_a": [], "k_d": [], "V": [],
        "D_x": [], "D_z": [], "mom_x_end": [], "mom_z_end": [],
    }
    for s, (ka, kd) in enumerate(SPECIES):
        ts = time.time()
        r = oracle.vacf(mask, u, 12 * D_B, ka, kd, args.steps, qmask=0b1010)
        D = oracle.d_of_t(r["Z"], r["V"])
        rec["k_a"].append(ka)
        rec["k_d"].append(kd)
        rec["V"].append(r["V"].tolist())
        rec["D_x"].append(D[0, grid].tolist())
        rec["D_z"].append(D[2, grid].tolist())
        rec["mom_x_end"].append(float(r["mom"][0, -1]))
        rec["mom_z_end"].append(float(r["mom"][2, -1]))
        with open(args.out + ".tmp", "w") as f:
            json.dump(rec, f, indent=1)
        os.replace(args.out + ".tmp", args.out)
        print(f"species {s} (k_a {ka}, k_d {kd}): {time.time() - ts:.0f}s, D_x/D_b(end) "
              f"{D[0, -1] / D_B:.6f}, D_z/D_b(end) {D[2, -1] / D_B:.6f}", flush=True)


if __name__ == "__main__":
    main()
