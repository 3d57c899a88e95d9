"""Learned surrogate for D_x(t)/D_b in random porous media, trained on runs of
the moment-propagation method itself (Sec. IV of the paper: predict the
time-dependent diffusion of species with known k_a, k_d in a given medium,
or extract k_a, k_d from D(t)).

Workload: 64^3 periodic Boolean sphere packs (radius R ~ U{4..10}, target
porosity ~ U[0.3, 0.7]), Peclet number Pe ~ U[0, 100] with the sample length
64 as length scale (Pe = 64 vbar / D_b, D_b = 1e-2), 8 species per medium
with k_a, k_d log-uniform in [1e-4, 1e-1]. Each (medium, Pe) group is one
batched propagation run; D_x(t) is sampled at 32 log-spaced times up to
D_b t / R^2 = 10. Features: porosity, specific surface N_I/N, Pe, log10 k_a,
log10 k_d, log10 t; target log10(D_x(t)/D_b).

The flow of a group is the BGK solution at a reference force rescaled to the
target Pe (creeping flow: the steady velocity is proportional to the force).
Every step runs in liblbmp's kernels; this module only orchestrates calls,
draws inputs and assembles feature rows.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs

N_LAT = 64
D_B = 0.01
SPECIES_PER_GROUP = 8
T_SAMPLES = 32
G_REF = 1e-6
DOMAIN = {  # training domain of the features, in feature order (fallback outside it)
    "porosity": (0.3, 0.7), "specific_surface": (0.0, 1.0), "peclet": (0.0, 100.0),
    "log10_ka": (-4.0, -1.0), "log10_kd": (-4.0, -1.0),
    # sampled times run from 1 to 10 R^2 / D_b, at most 1e5 (R <= 10)
    "log10_t": (0.0, 5.0),
}
MEDIUM_SHAPE = (N_LAT, N_LAT, N_LAT)  # Pe and N_I/N are defined on 64^3 samples


def group_params(seed: int) -> dict:
    """(medium, Pe, species) of one group, drawn from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    R = int(rng.integers(4, 11))
    phi = float(rng.uniform(0.3, 0.7))
    pe = float(rng.uniform(0.0, 100.0))
    lka = rng.uniform(-4, -1, SPECIES_PER_GROUP)
    lkd = rng.uniform(-4, -1, SPECIES_PER_GROUP)
    return {"seed": seed, "R": R, "phi": phi, "pe": pe, "k_a": 10.0 ** lka, "k_d": 10.0 ** lkd}


def sample_times(R: int) -> np.ndarray:
    """32 log-spaced integer times from 1 to 10 R^2 / D_b (unique)."""
    tmax = int(round(10 * R * R / D_B))
    t = np.unique(np.round(np.logspace(0, math.log10(tmax), T_SAMPLES)).astype(np.int64))
    return t


def run_groups(lb, groups: list[dict], log=None) -> tuple[np.ndarray, np.ndarray, dict]:
    """Runs a batch of groups in one batched handle; returns (X, y, info).

    X: (rows, 6) features, y: (rows,) log10(D_x/D_b)."""
    t0 = time.time()
    flows, species, meta = [], [], []
    for g in groups:
        mask = inputs.sphere_pack(N_LAT, g["R"], g["phi"], seed=g["seed"])
        ref = lb.lb_flow_solve(mask, 1.0, [G_REF, 0.0, 0.0], 1e-8, 200000)
        u = ref.velocity()
        fluid = mask == 0
        vbar = float(u[0][fluid].mean())
        target = g["pe"] * D_B / N_LAT
        scale = target / vbar if vbar > 0 else 0.0
        flow = lb.lb_flow_from_velocity(mask, u * scale)
        ref.free()
        _, nf, ni = flow.classes()
        flows.append(flow)
        species.append({"D_b": D_B, "k_a": g["k_a"], "k_d": g["k_d"]})
        meta.append({"porosity": nf / mask.size, "specific_surface": ni / mask.size,
                     "times": sample_times(g["R"])})
    tmax = int(max(m["times"][-1] for m in meta))
    t1 = time.time()
    mp = lb.mp_init(flows, species, lb.LBMP_FP32, tmax)
    lb.mp_step_n(mp, tmax)
    rows, ys = [], []
    for gi, (g, m) in enumerate(zip(groups, meta)):
        out = lb.mp_vacf(mp, gi, 0, int(m["times"][-1]) + 1)
        Dx = out["D"][:, 0, :]
        for s in range(SPECIES_PER_GROUP):
            d = Dx[s, m["times"]] / D_B
            for t, dv in zip(m["times"], d):
                if dv <= 0:
                    continue
                rows.append([m["porosity"], m["specific_surface"], g["pe"],
                             math.log10(g["k_a"][s]), math.log10(g["k_d"][s]), math.log10(t)])
                ys.append(math.log10(dv))
    mp.free()
    for f in flows:
        f.free()
    t2 = time.time()
    info = {"setup_s": t1 - t0, "propagation_s": t2 - t1, "steps": tmax}
    if log:
        log(f"groups {[g['seed'] for g in groups]}: flows {t1 - t0:.1f}s, propagation {t2 - t1:.1f}s "
            f"({tmax} steps)")
    return np.array(rows, dtype=np.float64), np.array(ys, dtype=np.float64), info


def build_dataset(lb, seeds, batch: int = 8, log=None):
    X, Y, infos = [], [], []
    for i in range(0, len(seeds), batch):
        x, y, info = run_groups(lb, [group_params(s) for s in seeds[i:i + batch]], log)
        X.append(x)
        Y.append(y)
        infos.append(info)
    return np.concatenate(X), np.concatenate(Y), infos


def query_features(shape, n_fluid: int, n_iface: int, peclet: float, k_a, k_d, times):
    """Feature rows (porosity, N_I/N, Pe, log10 k_a, log10 k_d, log10 t) of a
    query, species-major, or None when the network cannot answer it: a medium
    not of the training shape, a rate or time without a logarithm (k <= 0,
    t < 1), or any feature outside the training domain."""
    k_a = np.atleast_1d(np.asarray(k_a, dtype=np.float64))
    k_d = np.atleast_1d(np.asarray(k_d, dtype=np.float64))
    times = np.atleast_1d(np.asarray(times, dtype=np.float64))
    if tuple(shape) != MEDIUM_SHAPE:
        return None
    if not ((k_a > 0).all() and (k_d > 0).all() and (times >= 1).all() and np.isfinite(peclet)):
        return None
    n = float(np.prod(shape))
    feats = np.array([[n_fluid / n, n_iface / n, peclet, math.log10(a), math.log10(d), math.log10(t)]
                      for a, d in zip(k_a, k_d) for t in times])
    return feats if in_domain(feats).all() else None


def in_domain(features: np.ndarray) -> np.ndarray:
    f = np.atleast_2d(features)
    ok = np.ones(len(f), dtype=bool)
    for k, (lo, hi) in enumerate(DOMAIN.values()):
        ok &= (f[:, k] >= lo) & (f[:, k] <= hi)
    return ok


def train(lb, X: np.ndarray, Y: np.ndarray, epochs: int = 60, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0, log=None):
    """Trains a Surrogate on (X, Y) with a cosine learning-rate schedule."""
    import torch
    sg = lb.Surrogate(batch, seed=seed)
    mu, sd = X.mean(axis=0), X.std(axis=0)
    sd[sd == 0] = 1.0
    sg.set_normalization(mu, sd, float(Y.mean()), float(Y.std()))
    xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    yt = torch.tensor(Y, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    n = len(X)
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    k = 0
    losses = []
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(n).astype(np.int32), device="cuda")
        for i in range(steps_per_epoch):
            lr_k = 0.5 * lr * (1 + math.cos(math.pi * k / total))
            last = i == steps_per_epoch - 1
            loss = sg.train_step(xt, yt, perm[i * batch:], batch, lr_k, want_loss=last)
            k += 1
        losses.append(loss)
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: loss {loss:.4e}")
    return sg, losses


def evaluate(sg, X: np.ndarray, Y: np.ndarray) -> dict:
    """Relative error of D (not of log D) on held-out rows."""
    import torch
    xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    pred = sg.predict(xt)
    sg.sync()
    p = pred.cpu().numpy().astype(np.float64)
    rel = np.abs(10.0 ** (p - Y) - 1.0)
    out = {"p50": float(np.percentile(rel, 50)), "p95": float(np.percentile(rel, 95)),
           "max": float(rel.max()), "frac_within_2pct": float(np.mean(rel < 0.02)), "rows": int(len(Y))}
    # by decade of time: the long-time D_x of a flowing medium is its dispersion
    # coefficient, which the medium descriptors (porosity, surface) do not fix
    lt = X[:, 5]
    out["by_log10_t"] = {}
    for lo in range(0, 6):
        m = (lt >= lo) & (lt < lo + 1)
        if m.any():
            out["by_log10_t"][f"{lo}-{lo + 1}"] = {"rows": int(m.sum()), "p50": float(np.percentile(rel[m], 50)),
                                                    "p95": float(np.percentile(rel[m], 95))}
    return out


# Error-aware fallback: the held-out error of the network depends mostly on
# the time (late times carry the dispersion, which the medium descriptors do
# not fix) and on the Peclet number. Cells of half a decade in t by Pe band.
T_EDGES = np.arange(0.0, 6.01, 0.5)
PE_EDGES = np.array([0.0, 10.0, 30.0, 60.0, 100.0])


def error_cells(X: np.ndarray) -> np.ndarray:
    """Flat (log10 t, Pe) cell index of every feature row (edge cells absorb
    values beyond the edges)."""
    X = np.atleast_2d(X)
    ti = np.clip(np.searchsorted(T_EDGES, X[:, 5], side="right") - 1, 0, len(T_EDGES) - 2)
    pi = np.clip(np.searchsorted(PE_EDGES, X[:, 2], side="right") - 1, 0, len(PE_EDGES) - 2)
    return ti * (len(PE_EDGES) - 1) + pi


def error_table(X: np.ndarray, rel: np.ndarray, q: float = 95.0, min_rows: int = 50) -> np.ndarray:
    """q-th percentile of the relative error of D per (log10 t, Pe) cell from
    calibration rows; NaN (never trusted) where a cell has fewer than
    `min_rows` rows."""
    c = error_cells(X)
    tab = np.full((len(T_EDGES) - 1) * (len(PE_EDGES) - 1), np.nan)
    for k in np.unique(c):
        m = c == k
        if m.sum() >= min_rows:
            tab[k] = np.percentile(rel[m], q)
    return tab.reshape(len(T_EDGES) - 1, len(PE_EDGES) - 1)


def trusted(X: np.ndarray, table: np.ndarray, tol: float) -> np.ndarray:
    """Rows whose cell's calibrated error percentile is at most `tol`."""
    v = np.asarray(table, dtype=np.float64).ravel()[error_cells(X)]
    return ~np.isnan(v) & (v <= tol)


def split_groups(X: np.ndarray, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Row masks of two halves of the (medium, Pe) groups of X (a group's rows
    share porosity, specific surface and Pe), drawn at random."""
    _, g = np.unique(np.atleast_2d(X)[:, :3], axis=0, return_inverse=True)
    g = g.ravel()
    perm = np.random.default_rng(seed).permutation(g.max() + 1)
    first = np.isin(g, perm[: len(perm) // 2])
    return first, ~first


def query(lb, sg, mask: np.ndarray, peclet: float, k_a, k_d, times, velocity: np.ndarray | None = None,
          table: np.ndarray | None = None, tol: float = 0.02):
    """D_x(t)/D_b for species (k_a[i], k_d[i]) in a medium at Peclet `peclet`.

    In-domain queries are answered by the network; if any feature lies outside
    the training domain, or (with an error `table` from error_table) any
    (t, Pe) cell's calibrated error exceeds `tol`, the plain method runs
    instead (flow from `velocity` if given, otherwise the BGK solution
    rescaled to the Peclet number).
    Returns (D/D_b array (n_species, n_times), "surrogate" | "method")."""
    import torch
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    k_a = np.atleast_1d(np.asarray(k_a, dtype=np.float64))
    k_d = np.atleast_1d(np.asarray(k_d, dtype=np.float64))
    times = np.atleast_1d(np.asarray(times, dtype=np.int64))
    fluid = mask == 0
    # interface share from the library's own classification
    fl = lb.lb_flow_from_velocity(mask, np.zeros((3,) + mask.shape))
    _, nf, ni = fl.classes()
    fl.free()
    feats = query_features(mask.shape, nf, ni, peclet, k_a, k_d, times)
    ok = feats is not None
    if ok and table is not None:
        ok = bool(trusted(feats, table, tol).all())
    if ok:
        y = sg.predict(torch.tensor(feats, dtype=torch.float32, device="cuda"))
        sg.sync()
        return 10.0 ** y.cpu().numpy().reshape(len(k_a), len(times)), "surrogate"
    if velocity is None:
        ref = lb.lb_flow_solve(mask, 1.0, [G_REF, 0.0, 0.0], 1e-8, 200000)
        u = ref.velocity()
        ref.free()
        vbar = float(u[0][fluid].mean())
        velocity = u * ((peclet * D_B / mask.shape[2]) / vbar if vbar > 0 else 0.0)
    flow = lb.lb_flow_from_velocity(mask, velocity)
    tmax = int(times.max())
    mp = lb.mp_init(flow, {"D_b": D_B, "k_a": k_a, "k_d": k_d}, lb.LBMP_FP32, tmax)
    lb.mp_step_n(mp, tmax)
    out = lb.mp_vacf(mp, 0, 0, tmax + 1)
    mp.free()
    flow.free()
    return out["D"][:, 0, times] / D_B, "method"


def _batches_by_radius(seeds, batch):
    """Groups with the same sphere radius share a time horizon; batch them together."""
    by_r = {}
    for s in seeds:
        by_r.setdefault(group_params(s)["R"], []).append(s)
    out = []
    for r in sorted(by_r):
        ss = by_r[r]
        out += [ss[i:i + batch] for i in range(0, len(ss), batch)]
    return out


def main(argv=None):
    """Generate data with the batched method, train, evaluate on held-out media.

    Prints one JSON line: held-out relative error of D (p50/p95/max), the time
    per answered (species, t) query of the plain method and of the network,
    and their ratio."""
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser()
    ap.add_argument("--train-groups", type=int, default=512)
    ap.add_argument("--test-groups", type=int, default=64)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--save-data", metavar="NPZ", help="write the generated rows (and timings) to NPZ")
    ap.add_argument("--generate-only", action="store_true", help="stop after generating (and saving) the rows")
    ap.add_argument("--load-data", metavar="NPZ", nargs="+",
                    help="train and evaluate on the rows of one or more NPZ files (parts generated with "
                         "disjoint seeds are concatenated), no generation")
    args = ap.parse_args(argv)
    from . import lbmp
    lbmp.load_library()

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    if args.load_data:
        parts = [np.load(f) for f in args.load_data]
        Xtr = np.concatenate([d["Xtr"] for d in parts])
        Ytr = np.concatenate([d["Ytr"] for d in parts])
        Xte = np.concatenate([d["Xte"] for d in parts])
        Yte = np.concatenate([d["Yte"] for d in parts])
        t_gen = sum(float(d["t_gen"]) for d in parts)
        plain_s = sum(float(d["plain_s"]) for d in parts)
        answered = sum(int(d["answered"]) for d in parts)
        args.train_groups = sum(int(d["train_groups"]) for d in parts)
        args.test_groups = sum(int(d["test_groups"]) for d in parts)
    else:
        t0 = time.time()
        Xtr, Ytr = [], []
        for b in _batches_by_radius(list(range(args.seed, args.seed + args.train_groups)), args.batch):
            x, y, info = run_groups(lbmp, [group_params(s) for s in b], log)
            Xtr.append(x)
            Ytr.append(y)
        Xtr = np.concatenate(Xtr) if Xtr else np.zeros((0, 6))
        Ytr = np.concatenate(Ytr) if Ytr else np.zeros(0)
        t_gen = time.time() - t0
        # held-out media: new seeds; the plain method is timed on them
        Xte, Yte, plain_s, answered = [], [], 0.0, 0
        test_seeds = list(range(10 ** 6 + args.seed, 10 ** 6 + args.seed + args.test_groups))
        for b in _batches_by_radius(test_seeds, args.batch):
            ts = time.time()
            x, y, info = run_groups(lbmp, [group_params(s) for s in b], log)
            plain_s += time.time() - ts
            Xte.append(x)
            Yte.append(y)
            answered += len(y)
        Xte = np.concatenate(Xte) if Xte else np.zeros((0, Xtr.shape[1]))
        Yte = np.concatenate(Yte) if Yte else np.zeros(0)
        if args.save_data:
            np.savez(args.save_data, Xtr=Xtr, Ytr=Ytr, Xte=Xte, Yte=Yte, t_gen=t_gen, plain_s=plain_s,
                     answered=answered, train_groups=args.train_groups, test_groups=args.test_groups)
        if args.generate_only:
            print(json.dumps({"train_rows": int(len(Ytr)), "test_rows": int(len(Yte)), "generation_s": t_gen,
                              "plain_s": plain_s, "answered": answered}), flush=True)
            return
    if len(Yte) == 0:
        raise SystemExit("no held-out rows to evaluate on")
    t1 = time.time()
    sg, losses = train(lbmp, Xtr, Ytr, epochs=args.epochs, seed=args.seed, log=log)
    sg.sync()
    t_train = time.time() - t1
    ev = evaluate(sg, Xte, Yte)
    import torch
    xt = torch.tensor(Xte, dtype=torch.float32, device="cuda")
    sg.predict(xt)
    sg.sync()
    reps = 20
    ts = time.time()
    for _ in range(reps):
        sg.predict(xt)
    sg.sync()
    net_s = (time.time() - ts) / reps
    # error-aware fallback: calibrate the cell errors on half of the held-out
    # groups, measure what the gate lets through on the other half
    pred = sg.predict(torch.tensor(Xte, dtype=torch.float32, device="cuda"))
    sg.sync()
    rel = np.abs(10.0 ** (pred.cpu().numpy().astype(np.float64) - Yte) - 1.0)
    cal, tst = split_groups(Xte, args.seed)
    table = error_table(Xte[cal], rel[cal])
    gated = {"calibration_rows": int(cal.sum()), "test_rows": int(tst.sum()), "p95_table": table.tolist(),
             "t_edges": T_EDGES.tolist(), "pe_edges": PE_EDGES.tolist()}
    for tol in (0.02, 0.03, 0.05, 0.10):
        ok = trusted(Xte[tst], table, tol)
        r = rel[tst][ok]
        gated[f"tol_{tol:g}"] = {"answered": float(ok.mean()),
                                 "p50": float(np.percentile(r, 50)) if len(r) else None,
                                 "p95": float(np.percentile(r, 95)) if len(r) else None,
                                 "within_tol": float(np.mean(r <= tol)) if len(r) else None}
    res = {"metric": "surrogate D(t) error vs speedup", "train_rows": int(len(Ytr)),
           "test_rows": int(len(Yte)), "train_groups": args.train_groups, "test_groups": args.test_groups,
           "rel_err_D": ev, "final_train_loss": losses[-1],
           "plain_s_per_query": plain_s / answered, "surrogate_s_per_query": net_s / len(Yte),
           "speedup": (plain_s / answered) / (net_s / len(Yte)),
           "generation_s": t_gen, "training_s": t_train, "epochs": args.epochs, "gated": gated}
    print(json.dumps(res), flush=True)
    sg.free()


if __name__ == "__main__":
    main()
