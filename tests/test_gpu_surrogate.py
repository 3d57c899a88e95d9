"""Surrogate network kernels (BF16 MFMA, FP32 accumulation) vs the FP64 reference.

BF16 operands carry 8 significant bits, so outputs and gradients are compared
norm-wise: ||gpu - ref|| <= 2e-2 ||ref|| per tensor.
"""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1303_2470_amd import lbmp
    lbmp.load_library()
    return lbmp


def flat(params):
    return np.concatenate([p.reshape(-1) for p in params]).astype(np.float32)


def unflat(v, like):
    out, k = [], 0
    for p in like:
        out.append(v[k:k + p.size].reshape(p.shape))
        k += p.size
    return out


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_param_count(lb):
    sg = lb.Surrogate(64, seed=1)
    assert sg.n_params == 133633 == sum(p.size for p in mlp.init_params(0))
    p = sg.get_params()
    assert np.abs(p[: 256 * 6]).max() <= 1 / np.sqrt(6) + 1e-7
    sg.free()


@pytest.mark.parametrize("B", [32, 256, 1024])
def test_forward_matches_reference(lb, B):
    import torch
    params = mlp.init_params(5)
    rng = np.random.default_rng(B)
    x = rng.normal(size=(B, 6))
    sg = lb.Surrogate(1024, seed=0)
    sg.set_params(flat(params))
    assert np.array_equal(sg.get_params(), flat(params))
    y = sg.predict(torch.tensor(x, dtype=torch.float32, device="cuda"))
    sg.sync()
    yref, _ = mlp.forward(params, x)
    assert rel(y.cpu().numpy().astype(np.float64), yref) < 2e-2
    sg.free()


def test_predict_ragged_and_normalisation(lb):
    """n not a multiple of 32 nor of the batch size; z-scoring applied on the device."""
    import torch
    params = mlp.init_params(6)
    rng = np.random.default_rng(1)
    n = 1000
    x = rng.normal(size=(n, 6)) * 3 + 1
    mu, sd = x.mean(axis=0), x.std(axis=0)
    sg = lb.Surrogate(256, seed=0)
    sg.set_params(flat(params))
    sg.set_normalization(mu, sd, 0.5, 2.0)
    y = sg.predict(torch.tensor(x, dtype=torch.float32, device="cuda"))
    sg.sync()
    yref, _ = mlp.forward(params, (x - mu) / sd)
    assert rel(y.cpu().numpy(), 0.5 + 2.0 * yref) < 2e-2
    sg.free()


@pytest.mark.parametrize("B", [512, 8192])
def test_gradients_match_reference(lb, B):
    """Batch 8192 runs the hidden-layer GEMMs on the LDS-tiled kernel."""
    import torch
    params = mlp.init_params(7)
    rng = np.random.default_rng(3)
    x = rng.normal(size=(B, 6))
    t = np.sin(x[:, 0]) + 0.3 * x[:, 1] * x[:, 2]
    sg = lb.Surrogate(B, seed=0)
    sg.set_params(flat(params))
    g, loss = sg.gradients(torch.tensor(x, dtype=torch.float32, device="cuda"),
                           torch.tensor(t, dtype=torch.float32, device="cuda"), B)
    lref, gref = mlp.loss_and_grads(params, x, t)
    assert abs(loss / lref - 1) < 2e-2
    for a, b in zip(unflat(g, params), gref):
        assert rel(a, b) < 2e-2


def test_fused_predict_equals_layer_path(lb):
    """The fused inference kernel and the layer-by-layer forward of training
    do the same arithmetic: the loss from fused predictions equals the loss
    the training path reports (up to the order of the final mean)."""
    import torch
    params = mlp.init_params(8)
    rng = np.random.default_rng(4)
    B = 1024
    x = rng.normal(size=(B, 6))
    t = np.cos(x[:, 1]) - 0.2 * x[:, 3]
    sg = lb.Surrogate(B, seed=0)
    sg.set_params(flat(params))
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    tt = torch.tensor(t, dtype=torch.float32, device="cuda")
    _, loss = sg.gradients(xt, tt, B)
    y = sg.predict(xt)
    sg.sync()
    lf = float(((y - tt) ** 2).double().mean())
    assert abs(lf / loss - 1) < 1e-5
    sg.free()


def test_training_fits_smooth_function(lb):
    """Adam on the GPU drives the loss of a smooth 6-feature target down and
    tracks the FP64 reference trajectory for the first steps."""
    import torch
    rng = np.random.default_rng(11)
    n, B = 8192, 512
    x = rng.uniform(-1, 1, size=(n, 6))
    t = np.tanh(x[:, 0] + 0.5 * x[:, 1]) + 0.2 * x[:, 2] * x[:, 3] - 0.1 * x[:, 4] + 0.05 * x[:, 5]
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    tt = torch.tensor(t, dtype=torch.float32, device="cuda")
    params = mlp.init_params(2)
    sg = lb.Surrogate(B, seed=0)
    sg.set_params(flat(params))
    # first 5 steps on the first B rows vs the FP64 reference
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    ref = [p.copy() for p in params]
    for k in range(1, 6):
        sg.train_step(xt, tt, None, B, 1e-3)
        _, gr = mlp.loss_and_grads(ref, x[:B], t[:B])
        mlp.adam_step(ref, gr, m, v, k, 1e-3)
    got = unflat(sg.get_params(), params)
    for a, b, p0 in zip(got, ref, params):
        assert rel(a - p0, b - p0) < 5e-2       # the update itself, BF16 gradients
    losses = []
    for ep in range(30):
        perm = torch.tensor(rng.permutation(n).astype(np.int32), device="cuda")
        for i in range(n // B):
            l = sg.train_step(xt, tt, perm[i * B:], B, 1e-3, want_loss=(i == n // B - 1))
        losses.append(l)
    assert losses[-1] < 0.05 * float(np.var(t))
    y = sg.predict(xt)
    sg.sync()
    assert float(np.mean((y.cpu().numpy() - t) ** 2)) < 0.05 * float(np.var(t))
    sg.free()


def test_dataset_rows_and_fallback(lb):
    """One group of the surrogate workload (64^3 sphere pack): feature rows are
    finite and inside the training domain; a query outside the domain falls
    back to the method and equals a direct run."""
    from paper_1303_2470_amd import inputs, surrogate
    g = surrogate.group_params(5)
    g["R"] = 4                                     # short horizon for the test
    X, Y, info = surrogate.run_groups(lb, [g])
    assert X.shape[1] == 6 and len(X) == len(Y) > 8 * 20
    assert np.isfinite(X).all() and np.isfinite(Y).all()
    assert surrogate.in_domain(X).all()
    assert info["steps"] == surrogate.sample_times(4)[-1]
    sg = lb.Surrogate(256, seed=1)
    mask = inputs.sphere_pack(64, 4, 0.5, seed=3)   # the training media size
    u = inputs.random_velocity(mask, 0.005, seed=4)
    D, how = surrogate.query(lb, sg, mask, 10.0, [0.5], [0.01], [1, 10, 100], velocity=u)  # k_a out of domain
    assert how == "method"
    fl = lb.lb_flow_from_velocity(mask, u)
    mp = lb.mp_init(fl, {"D_b": surrogate.D_B, "k_a": [0.5], "k_d": [0.01]}, 32, 100)
    lb.mp_step_n(mp, 100)
    ref = lb.mp_vacf(mp, 0)["D"][0, 0, [1, 10, 100]] / surrogate.D_B
    assert np.allclose(D[0], ref, rtol=1e-6)
    D2, how2 = surrogate.query(lb, sg, mask, 10.0, [0.01, 0.001], [0.01, 0.05], [1, 10, 100])
    assert how2 == "surrogate" and D2.shape == (2, 3) and np.isfinite(D2).all()
    mp.free()
    sg.free()


def test_error_gated_fallback(lb):
    """With an error table, an in-domain query goes to the network only where
    every (t, Pe) cell's calibrated error is within the tolerance; otherwise
    the method runs and equals a direct run."""
    from paper_1303_2470_amd import inputs, surrogate
    sg = lb.Surrogate(256, seed=1)
    mask = inputs.sphere_pack(64, 4, 0.5, seed=3)   # the training media size
    u = inputs.random_velocity(mask, 0.005, seed=4)
    nt, npe = len(surrogate.T_EDGES) - 1, len(surrogate.PE_EDGES) - 1
    table = np.full((nt, npe), 0.01)
    table[2:, :] = 0.5                             # log10 t >= 1: not trusted at 5 %
    D, how = surrogate.query(lb, sg, mask, 10.0, [0.01], [0.02], [1, 3], velocity=u, table=table, tol=0.05)
    assert how == "surrogate" and D.shape == (1, 2)
    D, how = surrogate.query(lb, sg, mask, 10.0, [0.01], [0.02], [1, 30], velocity=u, table=table, tol=0.05)
    assert how == "method"
    fl = lb.lb_flow_from_velocity(mask, u)
    mp = lb.mp_init(fl, {"D_b": surrogate.D_B, "k_a": [0.01], "k_d": [0.02]}, 32, 30)
    lb.mp_step_n(mp, 30)
    ref = lb.mp_vacf(mp, 0)["D"][0, 0, [1, 30]] / surrogate.D_B
    assert np.allclose(D[0], ref, rtol=1e-6)
    table[:] = np.nan                              # no calibration: nothing is trusted
    _, how = surrogate.query(lb, sg, mask, 10.0, [0.01], [0.02], [1], velocity=u, table=table, tol=1.0)
    assert how == "method"
    mp.free()
    fl.free()
    sg.free()


def test_predict_orders_after_current_stream(lb):
    """Inputs produced by device kernels still running on the caller's stream:
    predict (on the handle's own stream) waits for them, and the caller's
    stream waits for the predictions."""
    import torch
    sg = lb.Surrogate(1024, seed=3)
    g = torch.Generator(device="cuda").manual_seed(1)
    x0 = torch.rand((4096, 6), device="cuda", generator=g)
    torch.cuda.synchronize()
    ref = sg.predict(x0.clone())
    sg.sync()
    ref = ref.cpu()
    # a slow producer on the current stream: x is written only after the matmuls
    y = torch.rand((2048, 2048), device="cuda", generator=g)
    for _ in range(30):
        y = (y @ y) / 2048.0
    x = x0 + 0.0 * y[:1, :6]
    out = sg.predict(x)
    got = (out * 1.0).cpu()          # consumed on the current stream without a sync
    assert torch.equal(got, ref)
    sg.free()


def test_training_graph_replays_equal_eager_steps(lb, monkeypatch):
    """The training step replays a captured graph (forward, backward, Adam);
    with eager work and synchronisations between replays, a change of batch
    size (a new capture) and varying learning rates, every step's parameters
    equal those of the same steps launched one kernel at a time."""
    import torch
    rng = np.random.default_rng(7)
    n = 4096
    x = torch.tensor(rng.normal(size=(n, 6)), dtype=torch.float32, device="cuda")
    y = torch.tensor(rng.normal(size=n), dtype=torch.float32, device="cuda")
    a = lb.Surrogate(1024, seed=11)
    monkeypatch.setenv("LBMP_SG_GRAPH", "0")
    b = lb.Surrogate(1024, seed=11)
    monkeypatch.delenv("LBMP_SG_GRAPH")
    for sg in (a, b):
        sg.set_normalization(np.zeros(6), np.ones(6), 0.0, 1.0)
    assert np.array_equal(a.get_params(), b.get_params())
    for step, B in enumerate([256, 256, 256, 512, 512, 256]):
        idx = torch.tensor(rng.permutation(n)[:B].astype(np.int32), device="cuda")
        lr = 1e-3 * (1 + step) / 3
        la = a.train_step(x, y, idx, B, lr, want_loss=step % 2 == 0)
        lb_ = b.train_step(x, y, idx, B, lr, want_loss=step % 2 == 0)
        assert la == lb_
        a.predict(x[:64])                           # eager work between replays
        a.sync()
        b.sync()
        assert np.array_equal(a.get_params(), b.get_params()), step
    a.free()
    b.free()
