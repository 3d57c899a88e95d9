"""Host logic of the surrogate's error-aware fallback: (log10 t, Pe) cells,
the calibrated error table, the trust decision and the split of held-out
rows by (medium, Pe) group. No GPU."""
import numpy as np

from paper_1303_2470_amd import surrogate as S


def rows(log_t, pe, phi=0.5, s=0.2):
    X = np.zeros((len(log_t), 6))
    X[:, 0], X[:, 1], X[:, 2], X[:, 5] = phi, s, pe, log_t
    return X


def test_cells_edges_and_clipping():
    nt, npe = len(S.T_EDGES) - 1, len(S.PE_EDGES) - 1
    c = S.error_cells(rows([0.0, 0.49, 0.5, 5.99, 7.0, -1.0], [0.0, 9.99, 10.0, 100.0, 250.0, 0.0]))
    ti, pi = c // npe, c % npe
    assert ti.tolist() == [0, 0, 1, nt - 1, nt - 1, 0]
    assert pi.tolist() == [0, 0, 1, npe - 1, npe - 1, 0]


def test_error_table_percentiles_and_sparse_cells():
    rng = np.random.default_rng(0)
    a = rows(np.full(200, 0.2), np.full(200, 5.0))        # cell (0, 0): errors 0 .. 0.199
    b = rows(np.full(10, 2.2), np.full(10, 50.0))         # too few rows
    X = np.concatenate([a, b])
    rel = np.concatenate([rng.permutation(np.arange(200) / 1000.0), np.zeros(10)])
    tab = S.error_table(X, rel, q=95.0, min_rows=50)
    assert tab.shape == (len(S.T_EDGES) - 1, len(S.PE_EDGES) - 1)
    assert np.isclose(tab[0, 0], np.percentile(np.arange(200) / 1000.0, 95))
    assert np.isnan(tab[4, 2]) and np.isnan(tab).sum() == tab.size - 1


def test_trusted():
    tab = np.full((len(S.T_EDGES) - 1, len(S.PE_EDGES) - 1), np.nan)
    tab[0, 0], tab[1, 0] = 0.01, 0.04
    X = rows([0.2, 0.7, 0.7, 3.0], [1.0, 1.0, 1.0, 1.0])
    assert S.trusted(X, tab, 0.02).tolist() == [True, False, False, False]
    assert S.trusted(X, tab, 0.05).tolist() == [True, True, True, False]
    assert not S.trusted(X, tab, np.inf)[3]                # NaN cells are never trusted


def test_split_groups_disjoint_whole_groups():
    parts = [rows(np.linspace(0, 4, 32), np.full(32, pe), phi=phi, s=s)
             for phi, s, pe in [(0.3, 0.1, 5.0), (0.4, 0.2, 20.0), (0.5, 0.3, 70.0), (0.6, 0.1, 40.0),
                                (0.3, 0.1, 50.0)]]
    X = np.concatenate(parts)
    a, b = S.split_groups(X, seed=3)
    assert (a ^ b).all() and a.any() and b.any()
    for k in range(len(parts)):
        m = slice(32 * k, 32 * (k + 1))
        assert a[m].all() or b[m].all()
    a2, _ = S.split_groups(X, seed=3)
    assert np.array_equal(a, a2)


def test_query_features_domain_guards():
    """Queries the network cannot answer give no feature rows (the method then
    runs): no logarithm for k_a = 0 or t = 0, times beyond the training
    horizon of 1e5 steps, a medium not 64^3, features outside the domain."""
    shape = (64, 64, 64)
    n = 64 ** 3
    ok = S.query_features(shape, int(0.5 * n), int(0.1 * n), 20.0, [1e-3, 1e-2], [1e-3, 1e-4], [1, 10, 1000])
    assert ok.shape == (6, 6) and S.in_domain(ok).all()
    assert np.allclose(ok[0], [0.5, 0.1, 20.0, -3.0, -3.0, 0.0], atol=1e-6)
    bad = [
        dict(k_a=[0.0], k_d=[1e-3], times=[10]),         # k_a = 0: allowed by the method, no log
        dict(k_a=[1e-3], k_d=[1e-3], times=[0]),         # t = 0
        dict(k_a=[1e-3], k_d=[1e-3], times=[200000]),    # beyond 1e5
        dict(k_a=[1e-3], k_d=[0.5], times=[10]),         # log10 k_d > -1
    ]
    for b in bad:
        assert S.query_features(shape, int(0.5 * n), int(0.1 * n), 20.0, **b) is None, b
    assert S.query_features((32, 32, 32), 16000, 3000, 20.0, [1e-3], [1e-3], [10]) is None
    assert S.query_features(shape, int(0.9 * n), int(0.1 * n), 20.0, [1e-3], [1e-3], [10]) is None
    assert S.query_features(shape, int(0.5 * n), int(0.1 * n), 150.0, [1e-3], [1e-3], [10]) is None
