"""Brute-force views of the tracer Markov chain behind moment propagation.

TEST INFRASTRUCTURE ONLY. These are independent formulations used to pin the
C oracle (``mp_oracle.c``); none of them shares code with it:

* ``dense_chain_vacf`` builds the full transition matrix of the chain on a tiny
  lattice and evaluates Z(m) = E[v(0) v(m)] by matrix powers.
* ``walkers`` samples the same chain with independent random walkers
  (the Brownian-dynamics alternative the paper mentions in Sec. II).
* ``slit_zchain_vacf`` is the exact one-dimensional reduction of a slit pore
  with laterally uniform flow: the lateral hops are internal to a layer.

The chain (Sec. II, Eqs. 7-11): a mobile tracer at fluid node r hops along a
D3Q19 link c_i with the probability p_i(r) of Eq. 8 when r + c_i is fluid;
at an interfacial node it adsorbs with p_a = k_a dt/dx, otherwise it stays;
an adsorbed tracer desorbs back to its node with p_d = k_d dt. The start is
distributed by the Boltzmann weights of Eq. 11. The velocity of a step is
the hop vector (zero for staying, adsorbing or desorbing).
"""
from __future__ import annotations

import itertools

import numpy as np

# D3Q19 moving links, listed independently of the C oracle's table
_LINKS = [c for c in itertools.product((-1, 0, 1), repeat=3) if 0 < sum(abs(v) for v in c) <= 2]
LINKS = np.array(_LINKS, dtype=np.int64)           # (18, 3) as (cx, cy, cz)
WEIGHTS = np.array([1.0 / 18 if sum(abs(v) for v in c) == 1 else 1.0 / 36 for c in _LINKS])


def link_probs(mask, u, lam, bmu=None):
    """p_i(r) for every node and the 18 links: array (18, nz, ny, nx).

    bmu: beta mu^ex(r) of a charged tracer; the diffusive part of a hop from
    r to r + c is then scaled by exp(-(bmu(r + c) - bmu(r)) / 2)."""
    mask = np.asarray(mask).astype(bool)
    nz, ny, nx = mask.shape
    if u is None:
        u = np.zeros((3,) + mask.shape)
    ux, uy, uz = u[0], u[1], u[2]
    usq = ux * ux + uy * uy + uz * uz
    p = np.zeros((18,) + mask.shape)
    for k, (cx, cy, cz) in enumerate(LINKS):
        # destination r + c fluid?
        dest_solid = np.roll(mask, shift=(-cz, -cy, -cx), axis=(0, 1, 2))
        cu = cx * ux + cy * uy + cz * uz
        diff = lam / 2
        if bmu is not None:
            dest_mu = np.roll(bmu, shift=(-cz, -cy, -cx), axis=(0, 1, 2))
            diff = lam / 2 * np.exp(-(dest_mu - bmu) / 2)
        pk = WEIGHTS[k] * (diff + 3 * cu + 4.5 * cu * cu - 1.5 * usq)
        p[k] = np.where(mask | dest_solid, 0.0, pk)
    return p


def interface_nodes(mask, nbhd=18):
    """Fluid nodes with a solid neighbour among the 18 (or 6) D3Q19 neighbours."""
    mask = np.asarray(mask).astype(bool)
    near = np.zeros_like(mask)
    for cx, cy, cz in LINKS:
        if nbhd == 6 and abs(cx) + abs(cy) + abs(cz) != 1:
            continue
        near |= np.roll(mask, shift=(-cz, -cy, -cx), axis=(0, 1, 2))
    return near & ~mask


def _states(mask, nbhd):
    mask = np.asarray(mask).astype(bool)
    fluid = np.flatnonzero(~mask.ravel())
    iface = np.flatnonzero(interface_nodes(mask, nbhd).ravel())
    return fluid, iface


def stationary_weights(mask, pa, pd, nbhd=18, bmu=None):
    """Eq. 11 weights over the chain's states: first the mobile states (fluid
    nodes in index order), then the adsorbed states (interfacial nodes in
    index order); with an excess chemical potential each state of node r
    carries the Boltzmann factor exp(-bmu(r))."""
    fluid, iface = _states(mask, nbhd)
    K = pa / pd
    if bmu is None:
        bf = np.ones(np.asarray(mask).size)
    else:
        bf = np.exp(-np.asarray(bmu, dtype=np.float64).ravel())
    w = np.concatenate([bf[fluid], K * bf[iface]])
    return w / w.sum()


def transition_matrix(mask, u, lam, pa, pd, nbhd=18, bmu=None):
    """The tracer chain on the states "mobile at a fluid node" (first N_F) and
    "adsorbed at an interfacial node" (next N_I), built link by link: M the
    transition matrix, B[g] its displacement-weighted version, C2[g] the
    conditional E[v_g^2 | state]. Returns (M, B, C2, n_fluid)."""
    mask = np.asarray(mask).astype(bool)
    nz, ny, nx = mask.shape
    fluid, iface = _states(mask, nbhd)
    nf, ni = len(fluid), len(iface)
    S = nf + ni
    mob = {int(n): k for k, n in enumerate(fluid)}
    ads = {int(n): nf + k for k, n in enumerate(iface)}
    p = link_probs(mask, u, lam, bmu).reshape(18, -1)
    M = np.zeros((S, S))
    B = np.zeros((3, S, S))
    C2 = np.zeros((3, S))          # E[v_g^2 | state]
    for n in fluid:
        s = mob[int(n)]
        z, rem = divmod(int(n), nx * ny)
        y, x = divmod(rem, nx)
        out = 0.0
        for k, (cx, cy, cz) in enumerate(LINKS):
            pk = p[k, n]
            if pk == 0.0:
                continue
            m = ((x + cx) % nx) + nx * (((y + cy) % ny) + ny * ((z + cz) % nz))
            t = mob[int(m)]
            M[s, t] += pk
            for g, c in enumerate((cx, cy, cz)):
                B[g, s, t] += pk * c
                C2[g, s] += pk * c * c
            out += pk
        if int(n) in ads:
            M[s, ads[int(n)]] += pa
            out += pa
        M[s, s] += 1.0 - out
    for n in iface:
        s = ads[int(n)]
        M[s, mob[int(n)]] += pd
        M[s, s] += 1.0 - pd
    return M, B, C2, nf


def dense_chain_vacf(mask, u, lam, pa, pd, steps, nbhd=18, bmu=None):
    """Z_g(m), m = 0..steps, from the explicit transition matrix.

    Z(0) = E[v(0)^2]; Z(m >= 1) = pi0^T B M^(m-1) b, where M is the transition
    matrix, B the displacement-weighted transition matrix and b = B 1.
    Returns (Z (3, steps+1), V (3,)).
    """
    M, B, C2, nf = transition_matrix(mask, u, lam, pa, pd, nbhd, bmu)
    pi0 = stationary_weights(mask, pa, pd, nbhd, bmu)
    b = B.sum(axis=2)
    V = pi0 @ b.T
    Z = np.zeros((3, steps + 1))
    Z[:, 0] = C2 @ pi0
    for g in range(3):
        row = pi0 @ B[g]                # E[v(0) 1{state at 1}]
        for m in range(1, steps + 1):
            Z[g, m] = row @ b[g]
            row = row @ M
    return Z, V


def dense_chain_uptake(mask, u, lam, pa, pd, steps, nbhd=18):
    """Mobile and adsorbed probability for t = 0..steps of the chain started
    uniformly on the mobile states (p_d = 0 allowed): pi_t = pi_0 M^t."""
    M, _, _, nf = transition_matrix(mask, u, lam, pa, pd, nbhd)
    pi = np.zeros(M.shape[0])
    pi[:nf] = 1.0 / nf
    mob, ads = np.zeros(steps + 1), np.zeros(steps + 1)
    for t in range(steps + 1):
        mob[t], ads[t] = pi[:nf].sum(), pi[nf:].sum()
        pi = pi @ M
    return mob, ads


def walkers(mask, u, lam, pa, pd, steps, n_walkers, seed, nbhd=18):
    """Monte Carlo estimate of v(0) v(m) and of the mean-square displacement.

    Walkers start from the Eq. 11 weights and follow the chain for ``steps``
    steps (link probabilities must be non-negative). Returns a dict with
    ``vv`` (3, steps) sample means of v_g(0) v_g(m), m = 0..steps-1, ``vv_se``
    their standard errors, ``msd`` (3, steps+1) the mean-square displacement
    about the sample-mean drift after n = 0..steps steps, and ``msd_se``.
    """
    mask = np.asarray(mask).astype(bool)
    nz, ny, nx = mask.shape
    rng = np.random.default_rng(seed)
    fluid, iface = _states(mask, nbhd)
    nf = len(fluid)
    pi0 = stationary_weights(mask, pa, pd, nbhd)
    st = rng.choice(len(pi0), size=n_walkers, p=pi0)
    is_ads = st >= nf
    node = np.empty(n_walkers, dtype=np.int64)
    node[~is_ads] = fluid[st[~is_ads]]
    node[is_ads] = iface[st[is_ads] - nf]
    iface_flag = np.zeros(mask.size, dtype=bool)
    iface_flag[iface] = True
    p = link_probs(mask, u, lam).reshape(18, -1)
    if (p < 0).any():
        raise ValueError("walkers need non-negative link probabilities")
    cum = np.cumsum(p, axis=0)                          # (18, N)
    disp = np.zeros((3, n_walkers))
    v0 = None
    vv = np.zeros((3, steps))
    vv_se = np.zeros((3, steps))
    msd = np.zeros((3, steps + 1))
    msd_se = np.zeros((3, steps + 1))
    for t in range(steps):
        r = rng.random(n_walkers)
        mob = ~is_ads
        k = (r[None, :] >= cum[:, node]).sum(axis=0)   # first link with r < cumulative p
        hop = mob & (k < 18)
        v = np.zeros((3, n_walkers))
        v[:, hop] = LINKS[k[hop]].T
        adsorb = mob & ~hop & iface_flag[node] & (r < cum[17, node] + pa)
        desorb = is_ads & (r < pd)
        if t == 0:
            v0 = v.copy()
        prod = v0 * v
        vv[:, t] = prod.mean(axis=1)
        vv_se[:, t] = prod.std(axis=1) / np.sqrt(n_walkers)
        z, rem = np.divmod(node, nx * ny)
        y, x = np.divmod(rem, nx)
        vi = v.astype(np.int64)
        moved = ((x + vi[0]) % nx) + nx * (((y + vi[1]) % ny) + ny * ((z + vi[2]) % nz))
        node = np.where(hop, moved, node)
        is_ads = (is_ads & ~desorb) | adsorb
        disp += v
        d = disp - disp.mean(axis=1, keepdims=True)
        d2 = d * d
        msd[:, t + 1] = d2.mean(axis=1)
        msd_se[:, t + 1] = d2.std(axis=1) / np.sqrt(n_walkers)
    return {"vv": vv, "vv_se": vv_se, "msd": msd, "msd_se": msd_se}


def slit_zchain_vacf(L, ux_profile, lam, pa, pd, steps, quantities=("x", "z")):
    """Exact 1D reduction of a slit of L fluid layers between solid planes.

    The flow is u = (ux(z), 0, 0) with ``ux_profile`` of length L. The states are
    the L mobile layers plus one adsorbed state on each wall layer. Hops with
    c_z = 0 keep the layer; hops into the walls are forbidden (Sec. II).
    Returns (Z (3, steps+1), V (3,)) for the requested directions
    (others left zero).
    """
    u = np.asarray(ux_profile, dtype=np.float64)
    # per-layer link probabilities, links into the walls removed
    p = np.zeros((18, L))
    for k, (cx, cy, cz) in enumerate(LINKS):
        cu = cx * u
        pk = WEIGHTS[k] * (lam / 2 + 3 * cu + 4.5 * cu * cu - 1.5 * u * u)
        dest = np.arange(L) + cz
        p[k] = np.where((dest >= 0) & (dest < L), pk, 0.0)
    up = p[LINKS[:, 2] == 1].sum(axis=0)
    down = p[LINKS[:, 2] == -1].sum(axis=0)
    wall = np.zeros(L, dtype=bool)
    wall[0] = wall[-1] = True
    K = pa / pd
    Zpart = L + 2 * K
    rho0 = np.full(L, 1.0 / Zpart)

    def step(X, Xa):
        Y = X * (1.0 - up - down - pa * wall)
        Y[1:] += X[:-1] * up[:-1]
        Y[:-1] += X[1:] * down[1:]
        Y += pd * Xa * wall
        Ya = np.where(wall, pa * X + (1 - pd) * Xa, 0.0)
        return Y, Ya

    Z = np.zeros((3, steps + 1))
    V = np.zeros(3)
    for g, name in enumerate(("x", "y", "z")):
        cg = LINKS[:, g]
        a = (p * cg[:, None]).sum(axis=0)
        V[g] = (rho0 * a).sum()
        Z[g, 0] = (rho0 * (p * (cg * cg)[:, None]).sum(axis=0)).sum()
        if name not in quantities:
            continue
        # first hop, weighted by its displacement, grouped by arrival layer
        X = np.zeros(L)
        for k in range(18):
            contrib = rho0 * p[k] * cg[k]
            dz = LINKS[k, 2]
            if dz == 0:
                X += contrib
            elif dz == 1:
                X[1:] += contrib[:-1]
            else:
                X[:-1] += contrib[1:]
        Xa = np.zeros(L)
        for t in range(1, steps + 1):
            Z[g, t] = (X * a).sum()
            X, Xa = step(X, Xa)
    return Z, V
