"""Writes ``c4_sphere256_dt.json``: FP64 oracle D(t), t = 0..200, of the full
256^3 porous workload (Boolean sphere pack, radius 8, porosity 0.4,
seed 2024) with a BGK flow at Pe = 10, for the species of smallest and
largest K = k_a/k_d of the workload's 16.

Calls only ``oracle`` and ``paper_1303_2470_amd.inputs`` (nothing comes from
the GPU path). The flow is BGK (tau = 1, Guo forcing, half-way bounce-back)
at the reference force (1e-6, 0, 0) after a fixed 1,000 steps from rest:
converging the 256^3 medium to a step change of 1e-10 takes about 5e4 steps,
some nine hours of the FP64 oracle on 8 cores, while a fixed number of steps
is reproduced by the GPU solver to rounding. The long-horizon check with a
converged flow is the 64^3 medium of make_c4_ref.py. The velocity is
rescaled to the mean fluid velocity Pe D_b / 256; species rates from
inputs.loguniform_rates(16, 1e-4, 1e-1, seed=2026).

Run: ``OMP_NUM_THREADS=8 python tests/golden/make_c4_256_ref.py`` (about 20
minutes on 8 cores, ~10 GB of memory).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1303_2470_amd import inputs  # noqa: E402

N, RADIUS, POROSITY, SEED, RATE_SEED = 256, 8, 0.4, 2024, 2026
D_B, PECLET, G_REF, FLOW_STEPS = 1e-2, 10.0, 1e-6, 1000
STEPS = 200
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_sphere256_dt.json")


def main():
    t0 = time.time()
    mask = inputs.sphere_pack(N, RADIUS, POROSITY, seed=SEED)
    fl = oracle.bgk(mask, 1.0, [G_REF, 0.0, 0.0], tol=0.0, max_steps=FLOW_STEPS, check_every=FLOW_STEPS + 1)
    if fl["steps"] != FLOW_STEPS:
        raise SystemExit(f"flow ran {fl['steps']} steps")
    fluid = mask == 0
    ux_ref = float(fl["u"][0][fluid].mean())
    u = fl["u"] * ((PECLET * D_B / N) / ux_ref)
    del fl
    print(f"flow: {FLOW_STEPS} steps, mean u_x {ux_ref:.12e}, {time.time() - t0:.0f}s", flush=True)
    ka, kd = inputs.loguniform_rates(16, 1e-4, 1e-1, seed=RATE_SEED)
    K = ka / kd
    picks = [int(np.argmin(K)), int(np.argmax(K))]
    rec = {"_about": __doc__.strip().splitlines()[0] + " Written by tests/golden/make_c4_256_ref.py.",
           "n": N, "radius": RADIUS, "porosity": POROSITY, "seed": SEED, "rate_seed": RATE_SEED,
           "D_b": D_B, "peclet": PECLET, "g_ref": G_REF, "flow_tol": 0.0, "flow_steps": FLOW_STEPS,
           "mean_ux_ref": ux_ref,
           "steps": STEPS, "species": picks, "k_a": [], "k_d": [], "V": [], "D": [], "mass_end": []}
    for s in picks:
        ts = time.time()
        r = oracle.vacf(mask, u, 12 * D_B, float(ka[s]), float(kd[s]), STEPS)
        D = oracle.d_of_t(r["Z"], r["V"])
        rec["k_a"].append(float(ka[s]))
        rec["k_d"].append(float(kd[s]))
        rec["V"].append(r["V"].tolist())
        rec["D"].append(D.tolist())
        rec["mass_end"].append(r["mass"][:, -1].tolist())
        print(f"species {s}: {time.time() - ts:.0f}s", flush=True)
    with open(OUT + ".tmp", "w") as f:
        json.dump(rec, f)
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
