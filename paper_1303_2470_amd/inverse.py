"""Adsorption and desorption rates from a measured D(t): the converse use of
the method named in the paper's conclusion (reference measurements of the
time-dependent diffusion coefficient in a controlled geometry fix k_a and k_d).

Batched refinement on the method itself: every round evaluates a grid of
(log10 k_a, log10 k_d) candidates as the species of one batched run (all of
them advance in the same launches), scores each by the root-mean-square
deviation of D(t) at the measured times, and shrinks the search box around
the best candidate. Every step runs in liblbmp's kernels; this module draws
the grids and compares curves.
"""
from __future__ import annotations

import math

import numpy as np


def _scale(D_target: np.ndarray) -> np.ndarray:
    """Per-direction scale of the residuals: the largest |D_target| it holds."""
    return np.abs(D_target).max(axis=-1, keepdims=True)


def residuals(D: np.ndarray, D_target: np.ndarray) -> np.ndarray:
    """Scaled deviations, one row per candidate (candidates in D's first axis)."""
    return ((D - D_target[None]) / _scale(D_target)[None]).reshape(len(D), -1)


def misfit(D: np.ndarray, D_target: np.ndarray) -> np.ndarray:
    """Root-mean-square scaled deviation of every candidate."""
    return np.sqrt(np.mean(residuals(D, D_target) ** 2, axis=1))


def refine(evaluate, D_target, bounds=((1e-4, 1e-1), (1e-4, 1e-1)), grid: int = 8,
           rounds: int = 3, zoom: float = 3.0, lm_iters: int = 30, h: float = 1e-4) -> dict:
    """Least-squares (log10 k_a, log10 k_d) within `bounds`.

    evaluate(k_a[n], k_d[n]) returns D[n, ...] shaped like D_target. First
    `rounds` of grid refinement (grid x grid candidates per batch, the box
    shrunk by `zoom` around the best); then Levenberg-Marquardt in log space,
    each iteration two batches: the centre with central differences of step h
    (5 candidates), then the damped Gauss-Newton step for six damping values.
    The grid finds the valley where k_a / k_d is fixed; the damped steps walk
    along it, where a shrinking grid alone can lose the minimum."""
    D_target = np.asarray(D_target, dtype=np.float64)
    lo = np.log10([bounds[0][0], bounds[1][0]])
    hi = np.log10([bounds[0][1], bounds[1][1]])
    center, half = (lo + hi) / 2, (hi - lo) / 2
    history = []

    def run(P):
        P = np.clip(P, lo, hi)
        R = residuals(np.asarray(evaluate(10.0 ** P[:, 0], 10.0 ** P[:, 1])), D_target)
        return P, R, np.sqrt(np.mean(R * R, axis=1))

    best_p, best_c = None, np.inf
    for _ in range(rounds):
        a = center[0] + np.linspace(-half[0], half[0], grid)
        d = center[1] + np.linspace(-half[1], half[1], grid)
        la, ld = np.meshgrid(a, d, indexing="ij")
        P, _, c = run(np.stack([la.ravel(), ld.ravel()], axis=1))
        i = int(np.argmin(c))
        if c[i] <= best_c:
            best_p, best_c = P[i], float(c[i])
        history.append({"stage": "grid", "log10_k": best_p.tolist(), "misfit": best_c})
        center, half = best_p, half / zoom

    p = best_p
    for _ in range(lm_iters):
        E = np.array([[0, 0], [h, 0], [-h, 0], [0, h], [0, -h]])
        _, R, c = run(p[None] + E)
        r0 = R[0]
        J = np.stack([(R[1] - R[2]) / (2 * h), (R[3] - R[4]) / (2 * h)], axis=1)
        A, g = J.T @ J, J.T @ r0
        steps = []
        for mu in (0.0, 1e-4, 1e-3, 1e-2, 1e-1, 1.0):
            try:
                dp = -np.linalg.solve(A + mu * np.trace(A) * np.eye(2), g)
            except np.linalg.LinAlgError:
                continue
            n = np.abs(dp).max()
            steps.append(dp if n <= 1.0 else dp / n)
        if not steps:
            break
        P, _, ct = run(p[None] + np.array(steps))
        i = int(np.argmin(ct))
        moved = np.abs(P[i] - p).max()
        if ct[i] < c[0]:
            p, best_c = P[i], float(ct[i])
        else:
            best_c = float(c[0])
        history.append({"stage": "lm", "log10_k": p.tolist(), "misfit": best_c})
        if ct[i] >= c[0] or moved < 1e-9:
            break
    return {"k_a": float(10.0 ** p[0]), "k_d": float(10.0 ** p[1]), "misfit": best_c, "history": history}


def path_evaluator(lb, flow, d_b: float, times, directions=(0,), precision: int = 64):
    """evaluate() for refine(): one batched run of the candidates on `flow`,
    D_g(t) for g in `directions` and t in `times`."""
    times = np.asarray(times, dtype=np.int64)
    tmax = int(times.max())
    dirs = list(directions)

    def evaluate(ka, kd):
        mp = lb.mp_init(flow, {"D_b": d_b, "k_a": ka, "k_d": kd}, precision, tmax)
        try:
            lb.mp_step_n(mp, tmax)
            return lb.mp_vacf(mp, 0, 0, tmax + 1)["D"][:, dirs][:, :, times]
        finally:
            mp.free()
    return evaluate


def fit(lb, flow, d_b: float, times, D_target, directions=(0,), precision: int = 64, **kw) -> dict:
    """(k_a, k_d) whose D_g(t) best matches D_target[len(directions), len(times)]."""
    D_target = np.asarray(D_target, dtype=np.float64).reshape(len(directions), len(times))
    return refine(path_evaluator(lb, flow, d_b, times, directions, precision), D_target, **kw)


def log_times(tmax: int, n: int = 24) -> np.ndarray:
    """About n log-spaced integer times in [1, tmax] (duplicates dropped)."""
    return np.unique(np.round(np.logspace(0, math.log10(tmax), n)).astype(np.int64))


def main(argv=None):
    """Fit (k_a, k_d) of a slit pore to a measured normal-direction D(t).

    The measurement file is JSON with L (fluid layers), D_b, times and D;
    prints one JSON line with the estimate and its iterations."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("measured")
    ap.add_argument("--k-a-range", type=float, nargs=2, default=(1e-4, 0.5))
    ap.add_argument("--k-d-range", type=float, nargs=2, default=(1e-5, 1e-1))
    args = ap.parse_args(argv)
    from . import inputs, lbmp
    lbmp.load_library()
    with open(args.measured) as f:
        meas = json.load(f)
    m = inputs.slit_mask(1, 1, int(meas["L"]) + 2)
    fl = lbmp.lb_flow_from_velocity(m, np.zeros((3,) + m.shape))
    r = fit(lbmp, fl, float(meas["D_b"]), np.array(meas["times"]), np.array(meas["D"]), directions=(2,),
            bounds=(tuple(args.k_a_range), tuple(args.k_d_range)))
    print(json.dumps(r))


if __name__ == "__main__":
    main()
