"""What the trained surrogate gains over the method (Sec. IV use: D(t) of
species of known k_a, k_d in a given medium): on held-out media, the time to
answer the same (species, t) queries with the network and with the plain
batched method, and the network's error against the method's answers.

A small version of the surrogate workload (64^3 sphere packs, radius 4, so the
time horizon is 1,600 steps): 12 training media, 4 held-out media, 8 species
each. The full-size evaluation (4,096 training runs, 512 held-out media) is a
separate, long GPU job (profiles/surrogate_eval.txt).
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1303_2470_amd import lbmp
    lbmp.load_library()
    return lbmp


def groups(seeds):
    from paper_1303_2470_amd import surrogate
    out = []
    for s in seeds:
        g = surrogate.group_params(s)
        g["R"] = 4                                   # shortest horizon of the workload
        out.append(g)
    return out


def test_surrogate_gain_on_held_out_media(lb):
    import torch
    from paper_1303_2470_amd import surrogate
    X, Y, _ = surrogate.run_groups(lb, groups(range(100, 112)))
    sg, losses = surrogate.train(lb, X, Y, epochs=60, batch=256, seed=3)
    assert losses[-1] < losses[0]
    # held-out media: the method's own answers, timed end to end (flows,
    # set-up, propagation, series)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xt, Yt, _ = surrogate.run_groups(lb, groups(range(10 ** 6 + 100, 10 ** 6 + 104)))
    torch.cuda.synchronize()
    t_method = time.perf_counter() - t0
    xt = torch.tensor(Xt, dtype=torch.float32, device="cuda")
    sg.predict(xt)
    sg.sync()
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        pred = sg.predict(xt)
    sg.sync()
    t_net = (time.perf_counter() - t0) / reps
    rel = np.abs(10.0 ** (pred.cpu().numpy().astype(np.float64) - Yt) - 1.0)
    speedup = t_method / t_net
    print(f"held-out queries {len(Yt)}: method {t_method:.3f} s, network {t_net * 1e6:.1f} us, "
          f"speed-up {speedup:.3g}; relative error p50 {np.median(rel):.3%}, p95 {np.percentile(rel, 95):.3%}")
    assert len(Yt) > 4 * 8 * 20
    assert speedup > 1e3
    assert np.isfinite(rel).all() and np.median(rel) < 0.2
    sg.free()
