"""ctypes front end of the FP64 C oracle (``mp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline of the benchmark call this; the product path never does.

Arrays follow the lattice convention ``(nz, ny, nx)`` with x fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i8 = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain IEEE double, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    c_int, c_long, c_double = ctypes.c_int, ctypes.c_long, ctypes.c_double
    vp = ctypes.c_void_p
    lib.orc_classify.argtypes = [c_int, c_int, c_int, _u8, c_int, _i8]
    lib.orc_links.argtypes = [c_int, c_int, c_int, _u8, vp, c_double, _dp]
    lib.orc_step.argtypes = [c_int, c_int, c_int, _i8, _dp, c_double, c_double, _dp, _dp, _dp, _dp]
    lib.orc_propagate.argtypes = [c_int, c_int, c_int, _u8, vp, c_double, c_double, c_double,
                                  c_int, c_long, _dp, _dp]
    lib.orc_vacf.argtypes = [c_int, c_int, c_int, _u8, vp, c_double, c_double, c_double, c_int,
                             c_long, c_int, _dp, _dp, _dp, _dp]
    lib.orc_bgk.argtypes = [c_int, c_int, c_int, _u8, c_double, _dp, c_double, c_long, c_int,
                            _dp, _dp, ctypes.POINTER(c_long), ctypes.POINTER(c_double)]
    lib.orc_uptake.argtypes = [c_int, c_int, c_int, _u8, vp, c_double, c_double, c_double, c_int,
                               c_long, _dp, _dp]
    lib.orc_links_charged.argtypes = [c_int, c_int, c_int, _u8, vp, c_double, vp, _dp]
    lib.orc_propagate_charged.argtypes = [c_int, c_int, c_int, _u8, vp, c_double, c_double, c_double,
                                          c_int, vp, c_long, _dp, _dp]
    lib.orc_vacf_charged.argtypes = [c_int, c_int, c_int, _u8, vp, c_double, c_double, c_double, c_int,
                                     vp, c_long, c_int, _dp, _dp, _dp, _dp]
    lib.orc_threads.argtypes = []
    lib.orc_set_threads.argtypes = [c_int]
    for f in ("orc_classify", "orc_links", "orc_step", "orc_propagate", "orc_vacf", "orc_bgk",
              "orc_uptake", "orc_threads", "orc_set_threads", "orc_links_charged",
              "orc_propagate_charged", "orc_vacf_charged"):
        getattr(lib, f).restype = c_int
    _lib = lib
    return lib


def threads() -> int:
    """OpenMP thread count the oracle runs on."""
    return int(_load().orc_threads())


def set_threads(n: int) -> int:
    """Run later oracle calls on n OpenMP threads; returns the new count."""
    return int(_load().orc_set_threads(int(n)))


def _mask(mask):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if m.ndim != 3:
        raise ValueError("mask must be (nz, ny, nx)")
    nz, ny, nx = m.shape
    return m, nx, ny, nz


def _vel(u, shape):
    if u is None:
        return None, None
    a = np.ascontiguousarray(u, dtype=np.float64)
    if a.shape != (3,) + shape:
        raise ValueError("velocity must be (3, nz, ny, nx)")
    return a, a.ctypes.data_as(ctypes.c_void_p)


def lambda_from(d_b: float | None = None, delta: float | None = None) -> float:
    """The paper's lambda from D_b = lambda c_s^2 / 4 (Sec. II) or from the rest
    stay probability delta = 1 - lambda/3 of a bulk node."""
    if (d_b is None) == (delta is None):
        raise ValueError("give exactly one of d_b, delta")
    return 12.0 * d_b if d_b is not None else 3.0 * (1.0 - delta)


def classify(mask, nbhd: int = 18) -> np.ndarray:
    """0 solid, 1 fluid, 2 interfacial fluid (Sec. II, Eq. 11 node classes)."""
    m, nx, ny, nz = _mask(mask)
    cls = np.zeros(m.shape, dtype=np.int8)
    _load().orc_classify(nx, ny, nz, m, nbhd, cls)
    return cls


def _bmu(bmu, shape):
    """beta mu^ex per node (charged tracers), or (None, None) for a neutral one."""
    if bmu is None:
        return None, None
    a = np.ascontiguousarray(bmu, dtype=np.float64)
    if a.shape != shape:
        raise ValueError("beta_mu_ex must be (nz, ny, nx)")
    return a, a.ctypes.data_as(ctypes.c_void_p)


def links(mask, u, lam: float, bmu=None) -> np.ndarray:
    """Link probabilities p_i(r) of Eq. 8, shape (19, nz, ny, nx); p_0 = 0.
    bmu: beta mu^ex(r) of a charged tracer (the Q term), or None."""
    m, nx, ny, nz = _mask(mask)
    ua, up = _vel(u, m.shape)
    ba, bp = _bmu(bmu, m.shape)
    p = np.zeros((19,) + m.shape)
    _load().orc_links_charged(nx, ny, nz, m, up, lam, bp, p)
    return p


def propagate(mask, u, lam: float, pa: float, pd: float, steps: int, X, Xa, nbhd: int = 18, bmu=None):
    """Propagate a (mobile, adsorbed) pair ``steps`` times (Eqs. 7, 9, 10)."""
    m, nx, ny, nz = _mask(mask)
    ua, up = _vel(u, m.shape)
    ba, bp = _bmu(bmu, m.shape)
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    Xa = np.array(Xa, dtype=np.float64, order="C", copy=True)
    _load().orc_propagate_charged(nx, ny, nz, m, up, lam, pa, pd, nbhd, bp, steps, X, Xa)
    return X, Xa


def vacf(mask, u, lam: float, pa: float, pd: float, steps: int, qmask: int = 15,
         nbhd: int = 18, bmu=None) -> dict:
    """Moment-propagation VACF for t = 0..steps (Eqs. 5, 11, 12).

    bmu: beta mu^ex(r) of a charged tracer (Q term of Eq. 8, Boltzmann factor
    of Eq. 11), or None for a neutral one.
    Returns a dict with ``Z`` (3, T+1), ``V`` (3,), ``mass`` (2, T+1) — mobile
    and adsorbed totals — and ``mom`` (3, T+1), the first-moment totals.
    """
    m, nx, ny, nz = _mask(mask)
    ua, up = _vel(u, m.shape)
    ba, bp = _bmu(bmu, m.shape)
    T1 = steps + 1
    Z = np.zeros(3 * T1)
    V = np.zeros(3)
    mass = np.zeros(2 * T1)
    mom = np.zeros(3 * T1)
    rc = _load().orc_vacf_charged(nx, ny, nz, m, up, lam, pa, pd, nbhd, bp, steps, qmask, Z, V, mass, mom)
    if rc != 0:
        raise ValueError("oracle rejected the input (no fluid node, or p_d <= 0)")
    return {"Z": Z.reshape(3, T1), "V": V, "mass": mass.reshape(2, T1),
            "mom": mom.reshape(3, T1)}


def uptake(mask, u, lam: float, pa: float, pd: float, steps: int, nbhd: int = 18) -> dict:
    """Out-of-equilibrium density propagation (Eqs. 7, 9, 10 with the density
    as the propagated quantity): uniform mobile start 1/N_F, nothing adsorbed;
    p_d = 0 allowed. Returns the mobile and adsorbed totals for t = 0..steps."""
    m, nx, ny, nz = _mask(mask)
    ua, up = _vel(u, m.shape)
    mob = np.zeros(steps + 1)
    ads = np.zeros(steps + 1)
    if _load().orc_uptake(nx, ny, nz, m, up, lam, pa, pd, nbhd, steps, mob, ads) != 0:
        raise ValueError("oracle rejected the input (no fluid node)")
    return {"mobile": mob, "adsorbed": ads}


def d_of_t(Z: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Discrete Eq. 3 with the long-time limit of Eq. 4 removed:
    D(n) = (Z(0) - V^2)/2 + sum_{m=1..n} (Z(m) - V^2), i.e. half the growth of
    the mean-square displacement (about the mean drift) between steps n and n+1."""
    Z = np.asarray(Z, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    c = Z - (V * V)[:, None]
    D = np.empty_like(c)
    D[:, 0] = 0.5 * c[:, 0]
    # compensated running sum
    for g in range(c.shape[0]):
        s, comp = D[g, 0], 0.0
        for t in range(1, c.shape[1]):
            v = c[g, t]
            tt = s + v
            comp += (s - tt) + v if abs(s) >= abs(v) else (v - tt) + s
            s = tt
            D[g, t] = s + comp
    return D


def bgk(mask, tau: float, g, tol: float = 1e-10, max_steps: int = 200000,
        check_every: int = 100) -> dict:
    """Steady D3Q19 BGK flow with Guo forcing and half-way bounce-back (Eq. 6)."""
    m, nx, ny, nz = _mask(mask)
    gg = np.ascontiguousarray(g, dtype=np.float64)
    u = np.zeros((3,) + m.shape)
    rho = np.zeros(m.shape)
    steps = ctypes.c_long(0)
    res = ctypes.c_double(0.0)
    rc = _load().orc_bgk(nx, ny, nz, m, tau, gg, tol, max_steps, check_every, u, rho,
                         ctypes.byref(steps), ctypes.byref(res))
    if rc < 0:
        raise ValueError("no fluid node")
    return {"u": u, "rho": rho, "steps": steps.value, "residual": res.value,
            "converged": rc == 0}
