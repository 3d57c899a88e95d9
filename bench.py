"""Benchmark: batched moment propagation with adsorption/desorption on one MI355X.

Workload (batched species and geometries): four slit pores of width
W = 16, 32, 48, 64 fluid layers with a 64 x 64 lateral extent (64 x 64 x (W+2)
lattices), each carrying 64 species with (k_a, k_d) drawn log-uniform in
[1e-4, 1e-1] from fixed seeds, D_b = 1e-2, in a Poiseuille flow at Peclet 10
(Pe = W vbar / D_b) from the BGK solver; FP32 propagation with FP64 sums.
One step advances all 256 (geometry, species) pairs by one time step, all
four propagated quantities and their adsorbed counterparts, and records the
VACF and conserved totals.

Prints one JSON line. ``value`` is fluid-node-species updates per second over
the timed steps (inputs resident on the GPU). ``roofline`` prices the
propagation kernel against the MI355X HBM peak; ``cpu_baseline`` times the
FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WIDTHS = (16, 32, 48, 64)
NXY = 64
N_SPECIES = 64
D_B = 0.01
PECLET = 10.0
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(lb, inputs):
    flows, species, nf, ni = [], [], [], []
    for i, W in enumerate(WIDTHS):
        mask = inputs.slit_mask(NXY, NXY, W + 2)
        g = inputs.poiseuille_force(PECLET, D_B, W)
        t0 = time.time()
        fl = lb.lb_flow_solve(mask, 1.0, [g, 0.0, 0.0], 1e-10, 400000)
        log(f"flow W={W}: {fl.steps} BGK steps, residual {fl.residual:.2e}, {time.time() - t0:.2f}s")
        ka, kd = inputs.loguniform_rates(N_SPECIES, 1e-4, 1e-1, seed=1000 + W)
        flows.append(fl)
        species.append({"D_b": D_B, "k_a": ka, "k_d": kd})
        _, f, n = fl.classes()
        nf.append(f)
        ni.append(n)
    return flows, species, nf, ni


def build_porous(lb):
    """The 256^3 periodic Boolean sphere pack (R = 8, porosity 0.4) with BGK
    flow rescaled to Pe = 10 on the sample length, 16 species with (k_a, k_d)
    log-uniform in [1e-4, 1e-1] (paper_1303_2470_amd.porous)."""
    from paper_1303_2470_amd import porous
    fl, sp = porous.build(lb, log=log)
    _, f, n = fl.classes()
    return [fl], [sp], [f], [n]


TRAFFIC_PATH = os.path.join(ROOT, "profiles", "mp_step_traffic.json")


def strip_comments(src: str) -> str:
    """C++ source without its comments and blank lines (string and character
    literals kept as they are), each line stripped of surrounding spaces."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":                                   # literal: copy up to its closing quote
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            while i < n and src[i] != "\n":
                i += 1
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = (l.strip() for l in "".join(out).splitlines())
    return "\n".join(l for l in lines if l)


def kernel_source_sha() -> str:
    """Hash of the propagation kernels' code (comments and layout ignored), the
    key under which measured traffic is recorded."""
    src = open(os.path.join(ROOT, "paper_1303_2470_amd", "csrc", "mp.hip"), encoding="utf-8").read()
    return hashlib.sha256(strip_comments(src).encode()).hexdigest()


def traffic_record(key: str):
    """Measured HBM bytes per launch of the propagation kernel, if taken on the
    current kernel source with the same workload and tile choice
    ("workload:variant,K,species per block") as this run
    (profiles/mp_step_traffic.json holds one entry per measured key)."""
    if not os.path.exists(TRAFFIC_PATH):
        return None
    rec = json.load(open(TRAFFIC_PATH))
    if rec.get("kernel_source_sha256") != kernel_source_sha():
        return None
    ent = rec.get("tiles", {}).get(key)
    return ent.get("bytes_per_launch") if ent else None


KERNELS = {0: ("direct", "k_mp_step"), 1: ("lds-box", "k_mp_step_box"), 2: ("z-march", "k_mp_march"),
           3: ("lds-dma", "k_mp_dma"), 4: ("lds-dma-zpair", "k_mp_dma"),
           5: ("lds-dma-rows", "k_mp_dma"), 6: ("lds-dma-zpair-rows", "k_mp_dma"),
           7: ("lds-dma-zpair-lanes", "k_mp_dma"), 8: ("gathered-chunks", "k_mp_gather")}


def rocprof_summary(root: str) -> dict:
    """Per-kernel summary of rocprofv3 CSV output under `root`: dispatch count
    and the median per dispatch of its duration and of every counter."""
    import csv
    import glob
    from collections import defaultdict
    out = {}
    for f in glob.glob(os.path.join(root, "**", "*kernel_stats.csv"), recursive=True):
        out.setdefault("kernel_stats", []).extend(
            {k: r[k] for k in ("Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage") if k in r}
            for r in csv.DictReader(open(f)))
    for f in glob.glob(os.path.join(root, "**", "*kernel_trace.csv"), recursive=True):
        d = defaultdict(list)
        for r in csv.DictReader(open(f)):
            d[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        out["kernel_trace"] = {k: {"n": len(v), "median_ns": float(np.median(v)), "mean_ns": float(np.mean(v))}
                               for k, v in d.items()}
    for f in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        d = defaultdict(lambda: defaultdict(list))
        for r in csv.DictReader(open(f)):
            d[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        cc = out.setdefault("counters", {})
        for k, v in d.items():
            cc.setdefault(k, {}).update({c: {"n": len(x), "median": float(np.median(x))} for c, x in v.items()})
    return out


def traffic_from_counters(root: str, copy_bytes: int) -> dict:
    """HBM bytes per launch of the DMA propagation kernel from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for the plain copy of `copy_bytes` bytes in the same directory tree."""
    summ = rocprof_summary(root)["counters"]

    def pick(name_part, counter):
        vals = [v[counter]["median"] for k, v in summ.items() if name_part in k and counter in v]
        return vals[0] if vals else None
    kern = os.environ.get("LBMP_KERNEL", "k_mp_dma")
    fk, wk = pick(kern, "FETCH_SIZE"), pick(kern, "WRITE_SIZE")
    # the copy kernel: the only other kernel profiled in those runs
    cf = [v["FETCH_SIZE"]["median"] for k, v in summ.items() if "k_mp" not in k and "FETCH_SIZE" in v]
    cw = [v["WRITE_SIZE"]["median"] for k, v in summ.items() if "k_mp" not in k and "WRITE_SIZE" in v]
    f_scale = copy_bytes / (max(cf) * 1024.0)
    w_scale = copy_bytes / (max(cw) * 1024.0)
    return {"kernel": kern, "tile": os.environ.get("LBMP_TILE"),
            "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
            "copy_bytes": copy_bytes, "fetch_scale": f_scale, "write_scale": w_scale,
            "bytes_per_launch": fk * 1024.0 * f_scale + wk * 1024.0 * w_scale}


def cpu_baseline(inputs, steps: int):
    """FP64 oracle on the widest slit of the workload, one species, `steps` steps."""
    import oracle
    oracle.build()
    W = WIDTHS[-1]
    mask = inputs.slit_mask(NXY, NXY, W + 2)
    ka, kd = inputs.loguniform_rates(N_SPECIES, 1e-4, 1e-1, seed=1000 + W)
    g = inputs.poiseuille_force(PECLET, D_B, W)
    # the flow is set up outside the timed part, as on the GPU
    col = oracle.bgk(inputs.slit_mask(1, 1, W + 2), 1.0, [g, 0, 0], 1e-10, 400000)
    u = np.broadcast_to(col["u"], (3, W + 2, NXY, NXY)).copy()
    t0 = time.time()
    ref = oracle.vacf(mask, u, 12 * D_B, float(ka[0]), float(kd[0]), steps)
    el = time.time() - t0
    nf = NXY * NXY * W
    cores = oracle.threads()
    # the same oracle on one core, over a shorter sample
    steps1 = max(1, steps // 15)
    oracle.set_threads(1)
    try:
        t1 = time.time()
        oracle.vacf(mask, u, 12 * D_B, float(ka[0]), float(kd[0]), steps1)
        el1 = time.time() - t1
    finally:
        oracle.set_threads(cores)
    return {"value": nf * steps / el, "unit": "fluid-node-species updates/s",
            "cores": cores, "kind": "oracle",
            "sample": f"64x64x{W + 2} slit (widest of the workload), 1 species, {steps} steps, "
                      f"FP64 stay form incl. its per-run set-up; {el:.1f}s",
            "one_core": {"value": nf * steps1 / el1, "cores": 1,
                         "sample": f"same slit and species, {steps1} steps on one thread; {el1:.1f}s"},
            "_D": oracle.d_of_t(ref["Z"], ref["V"])}


def d_error_vs_oracle(D_gpu: np.ndarray, D_ref: np.ndarray) -> dict:
    """Largest relative D(t) error over every recorded time and direction,
    |D - D_ref| / max(|D_ref|, 1e-2 D_b) (FP32 storage resolves D to about
    2^-24 Z(0)), against the 1e-5 tolerance."""
    err = np.abs(D_gpu - D_ref) / np.maximum(np.abs(D_ref), 1e-2 * D_B)
    return {"max_rel": float(err.max()), "tolerance": 1e-5, "times": int(D_ref.shape[-1]),
            "directions": int(D_ref.shape[0]),
            "case": "species 0 of the widest slit (W=64), t = 0 .. the oracle leg's steps, x/y/z"}


def sequential_compare(lb, flows, species, steps: int, warmup: int) -> dict:
    """The batched run against one run per (geometry, species) pair, each a
    handle of its own advancing the same number of steps through mp_step_n
    (graph replay), wall clock around the queued steps."""
    def timed(mp):
        lb.mp_step_n(mp, warmup)
        mp.stream.synchronize()
        t0 = time.perf_counter()
        lb.mp_step_n(mp, steps)
        mp.stream.synchronize()
        return time.perf_counter() - t0

    mp = lb.mp_init(flows, species, lb.LBMP_FP32, warmup + steps)
    tb = timed(mp)
    mp.free()
    ts, runs = 0.0, 0
    for fl, sp in zip(flows, species):
        for s in range(len(sp["k_a"])):
            one = {"D_b": sp["D_b"], "k_a": sp["k_a"][s:s + 1], "k_d": sp["k_d"][s:s + 1]}
            mp = lb.mp_init(fl, one, lb.LBMP_FP32, warmup + steps)
            ts += timed(mp)
            mp.free()
            runs += 1
    return {"metric": "batched vs sequential moment propagation", "steps": steps, "warmup": warmup,
            "batched_ms_per_step": tb / steps * 1e3, "sequential_runs": runs,
            "sequential_ms_per_step": ts / steps * 1e3, "speedup": ts / tb}


def surrogate_throughput(lb, n: int, batch_max: int, train_batch: int, reps: int) -> dict:
    """Inference and training-step throughput of the BF16-MFMA network on
    random inputs (weights from its own initialisation): samples/s and the
    GEMM work per second against the dense BF16 MFMA peak."""
    import torch
    # flop per sample: 2 x (multiply-adds of 6->256, 256->256, 256->256, 256->1)
    fwd = 2 * (6 * 256 + 256 * 256 + 256 * 256 + 256)
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.rand((n, 6), device="cuda", generator=g, dtype=torch.float32)
    sg = lb.Surrogate(batch_max, seed=1)
    out = sg.predict(x)
    sg.sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        sg.predict(x, out)
    sg.sync()
    tp = (time.perf_counter() - t0) / reps
    sg.free()
    peak = 2.5e15
    res = {"metric": "surrogate throughput", "predict_rows": n, "predict_chunk": batch_max,
           "predict_s": tp, "predict_samples_per_s": n / tp, "predict_tflops": fwd * n / tp / 1e12,
           "predict_frac_bf16_peak": fwd * n / tp / peak, "peak_tflops_bf16": peak / 1e12, "train": []}
    for tb in (train_batch, 8 * train_batch):
        st = lb.Surrogate(tb, seed=1)
        y = torch.rand((tb,), device="cuda", generator=g, dtype=torch.float32)
        xt = x[:tb].contiguous()
        st.train_step(xt, y, None, tb, 1e-4)
        st.sync()
        t0 = time.perf_counter()
        for _ in range(reps * 10):
            st.train_step(xt, y, None, tb, 1e-4)
        st.sync()
        tt = (time.perf_counter() - t0) / (reps * 10)
        st.free()
        res["train"].append({"batch": tb, "step_s": tt, "samples_per_s": tb / tt,
                             "tflops": 3 * fwd * tb / tt / 1e12, "frac_bf16_peak": 3 * fwd * tb / tt / peak})
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=1500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("slits", "porous256"), default="slits",
                    help="slits: the batched-slit configuration (default); porous256: the 256^3 sphere "
                         "pack with 16 species (no CPU baseline)")
    ap.add_argument("--surrogate", action="store_true",
                    help="only time the surrogate network: inference on 2^20 rows, training steps")
    ap.add_argument("--sequential", action="store_true",
                    help="only compare the batched slit run with one run per (geometry, species) pair")
    ap.add_argument("--copy-bandwidth", action="store_true",
                    help="only time device-to-device copies (torch) from 16 MiB to 4 GiB: the bandwidth a "
                         "streaming kernel can reach on this GPU, read + write bytes per second")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized buffer 5 times (known traffic, to scale HBM counters)")
    ap.add_argument("--rocprof-summary", metavar="DIR", help="only summarise rocprofv3 CSV output under DIR")
    ap.add_argument("--traffic-record", metavar="DIR",
                    help="only write profiles/mp_step_traffic.json from FETCH_SIZE / WRITE_SIZE runs of the "
                         "bench and of --copy-calibration 1024 under DIR")
    args = ap.parse_args()
    if args.rocprof_summary:
        print(json.dumps(rocprof_summary(args.rocprof_summary), indent=1))
        return
    if args.traffic_record:
        # one entry per workload and tile (--workload, LBMP_TILE of the counter runs); entries of an
        # older kernel source are dropped
        ent = traffic_from_counters(args.traffic_record, 1024 << 20)
        rec = json.load(open(TRAFFIC_PATH)) if os.path.exists(TRAFFIC_PATH) else {}
        if rec.get("kernel_source_sha256") != kernel_source_sha():
            rec = {"kernel": "k_mp_dma", "kernel_source_sha256": kernel_source_sha(),
                   "key": "sha256 of paper_1303_2470_amd/csrc/mp.hip with comments and blank lines removed",
                   "tiles": {}}
        ent["workload"] = args.workload
        rec["tiles"][f'{args.workload}:{ent["tile"]}'] = ent
        with open(TRAFFIC_PATH, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(ent))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the batched workload is one GPU's share "
              f"(species/geometry sharding needs no exchange); --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1303_2470_amd import inputs, lbmp
    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    if args.copy_bandwidth:
        out = []
        for mib in (16, 64, 128, 256, 512, 1024, 2048, 4096):
            n = mib << 20
            a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            reps = 20 if mib <= 256 else 5
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                b.copy_(a)
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            out.append({"bytes_per_buffer": n, "ms": ms, "read_plus_write_GBs": 2 * n / ms / 1e6})
            del a, b
        print(json.dumps({"copy_bandwidth": out}))
        return
    if args.copy_calibration:
        n = args.copy_calibration << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "launches": 5}))
        return
    lbmp.load_library()
    if args.surrogate:
        print(json.dumps(surrogate_throughput(lbmp, 1 << 20, 1 << 16, 1024, 20)), flush=True)
        return
    if args.sequential:
        flows, species, nf, ni = build_workload(lbmp, inputs)
        print(json.dumps(sequential_compare(lbmp, flows, species, args.steps, args.warmup)), flush=True)
        return
    if args.workload == "slits":
        flows, species, nf, ni = build_workload(lbmp, inputs)
        n_species = N_SPECIES
        lat_nodes = sum(NXY * NXY * (W + 2) for W in WIDTHS)
        workload = ("batched slits W=16,32,48,64 fluid layers x 64x64 lateral, 64 species each (k_a,k_d "
                    "log-uniform 1e-4..1e-1), D_b=1e-2, Poiseuille Pe=10, FP32 propagation + FP64 sums")
    else:
        flows, species, nf, ni = build_porous(lbmp)
        from paper_1303_2470_amd import porous
        n_species = porous.N_SPECIES
        lat_nodes = porous.N ** 3
        workload = ("256^3 periodic Boolean sphere pack R=8 porosity 0.4, 16 species (k_a,k_d log-uniform "
                    "1e-4..1e-1), D_b=1e-2, BGK flow at Pe=10, FP32 propagation + FP64 sums")
        args.no_cpu_baseline = True
    # warmup, the timed steps (graph replay, the production path), then the
    # same number of steps with every propagation-kernel launch bracketed by
    # HIP events (the kernel's own duration for the roofline)
    total = args.warmup + 2 * args.steps
    t0 = time.time()
    mp = lbmp.mp_init(flows, species, lbmp.LBMP_FP32, total)
    log(f"mp_init (incl. tile tuning): {time.time() - t0:.2f}s")
    st = lbmp.mp_stats(mp, 0)
    lbmp.mp_step_n(mp, args.warmup)
    mp.stream.synchronize()
    torch.cuda.synchronize()
    # timed region: K steps queued by mp_step_n (captured graphs replayed on
    # the handle's stream), HIP events recorded on that stream around them
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(mp.stream)
    lbmp.mp_step_n(mp, args.steps)
    e1.record(mp.stream)
    e1.synchronize()
    torch.cuda.synchronize()
    tot_ms = e0.elapsed_time(e1)
    k_ms, prof_ms = lbmp.mp_profile_steps(mp, args.steps)
    torch.cuda.synchronize()
    upd_per_step = sum(f * n_species for f in nf)
    value = upd_per_step * args.steps / (tot_ms / 1e3)
    # algorithmic bytes per launch: every quantity of every (node, species) read
    # and written once (4 quantities x 4 B x 2), the same for the adsorbed
    # quantities of interfacial nodes, and 16 B of flow data per fluid node
    alg = sum(n_species * (32 * f + 32 * n) + 16 * f for f, n in zip(nf, ni))
    k_avg_s = k_ms / 1e3 / args.steps
    achieved = alg / k_avg_s / 1e9
    traffic = traffic_record(f'{args.workload}:{st["kernel_variant"]},{st["tile_k"]},{st["species_per_block"]}')
    # accuracy and invariants of this run
    out = lbmp.mp_vacf(mp, len(flows) - 1, total, 1)
    mass_err = float(np.abs(out["mass"].sum(axis=1) - 1).max())
    mp.free()
    D_first = None
    if not args.no_cpu_baseline and args.workload == "slits":
        # the oracle check, independent of --steps: the same workload on a
        # handle of its own, cpu_steps steps through mp_step_n, outside the
        # timed region; D(t) of the widest slit's species 0 at every time
        mpc = lbmp.mp_init(flows, species, lbmp.LBMP_FP32, args.cpu_steps)
        lbmp.mp_step_n(mpc, args.cpu_steps)
        D_first = lbmp.mp_vacf(mpc, len(flows) - 1, 0, args.cpu_steps + 1)["D"][0]
        mpc.free()
    res = {
        "metric": "moment-prop node-species updates/s",
        "value": value,
        "unit": "fluid-node-species updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tot_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload,
                   "geometries": len(flows), "species_per_geometry": n_species,
                   "fluid_nodes": int(sum(nf)), "interface_nodes": int(sum(ni)),
                   "lattice_nodes": int(lat_nodes),
                   "lattice_node_species_updates_per_s": lat_nodes * n_species * args.steps / (tot_ms / 1e3),
                   "tile": {"K": st["tile_k"], "species_per_block": st["species_per_block"],
                            "variant": KERNELS[st["kernel_variant"]][0]}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic if st["kernel_variant"] >= 3 else None,
                     "kernel": KERNELS[st["kernel_variant"]][1], "kernel_avg_ms": k_avg_s * 1e3,
                     "algorithmic_bytes_per_launch": alg,
                     "timing": "achieved = algorithmic bytes / kernel_avg_ms (HIP events around every "
                               "launch of the propagation kernel, a second run of `steps` steps); "
                               "ms_per_step and value: graph replay of mp_step_n",
                     "event_bracketed_ms_per_step": prof_ms / args.steps},
        "mass_error_max": mass_err,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(inputs, args.cpu_steps)
        D_ref = cb.pop("_D")
        res["cpu_baseline"] = cb
        if D_first is not None:
            res["d_error_vs_oracle"] = d_error_vs_oracle(D_first, D_ref)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
