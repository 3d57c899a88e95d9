"""Python binding of liblbmp (include/lbmp.h): argument marshalling only.

Every step of the method runs in the HIP library. PyTorch provides device
memory (workspaces are uint8 tensors on the GPU) and streams. Importing this
module loads ``liblbmp.so`` and raises if it is missing or the GPU is absent:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmp.so")

LBMP_OK = 0
STATUS = {0: "LBMP_OK", -1: "LBMP_EINVAL", -2: "LBMP_EDEVICE", -3: "LBMP_ENOMEM",
          -4: "LBMP_ENOTCONV", -5: "LBMP_EPROB", -6: "LBMP_ESTATE", -7: "LBMP_ENUMERIC"}
LBMP_FP32, LBMP_FP64 = 32, 64


class LbmpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("periodic", ctypes.c_int * 3), ("solid", ctypes.c_void_p),
                ("iface_nbhd", ctypes.c_int)]


class Species(ctypes.Structure):
    _fields_ = [("D_b", ctypes.c_double), ("Delta", ctypes.c_double), ("n_species", ctypes.c_int),
                ("k_a", ctypes.c_void_p), ("k_d", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_fluid", ctypes.c_int64), ("n_iface", ctypes.c_int64),
                ("lambda_", ctypes.c_double), ("min_p", ctypes.c_double),
                ("max_cell_peclet", ctypes.c_double), ("min_stay", ctypes.c_double),
                ("mean_velocity", ctypes.c_double * 3), ("tile_k", ctypes.c_int),
                ("species_per_block", ctypes.c_int), ("kernel_variant", ctypes.c_int)]


EXPORTS = ["lbmp_last_error", "lbmp_version", "lb_flow_workspace_bytes", "lb_flow_solve",
           "lb_flow_solve_static", "lb_flow_static_max_nodes", "lb_flow_from_velocity", "lb_flow_velocity", "lb_flow_classes", "lb_flow_free",
           "mp_workspace_bytes", "mp_init", "mp_init_charged", "mp_step_n", "mp_vacf", "mp_steps_done", "mp_stats",
           "mp_uptake_init", "mp_uptake",
           "mp_state", "mp_profile_steps", "mp_checkpoint_bytes", "mp_save", "mp_load", "mp_free",
           "sg_param_count", "sg_workspace_bytes",
           "sg_create", "sg_set_params", "sg_get_params", "sg_set_normalization", "sg_train_step",
           "sg_gradients", "sg_predict", "sg_sync", "sg_free"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbmp.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    # PyTorch-ROCm ships its own HIP runtime; load it first so that liblbmp
    # binds to the same runtime that owns the workspaces and streams
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "lbmp_last_error": ([], ctypes.c_char_p),
        "lbmp_version": ([], ctypes.c_char_p),
        "lb_flow_workspace_bytes": ([P(Geometry), P(sz), P(sz)], i32),
        "lb_flow_solve": ([P(Geometry), dbl, P(dbl), dbl, i64, i32, vp, sz, vp, sz, vp, P(vp),
                           P(i64), P(dbl)], i32),
        "lb_flow_solve_static": ([P(Geometry), dbl, P(dbl), dbl, i64, i32, vp, sz, vp, P(vp), P(i64),
                                  P(dbl)], i32),
        "lb_flow_static_max_nodes": ([], i64),
        "lb_flow_from_velocity": ([P(Geometry), vp, vp, sz, vp, P(vp)], i32),
        "lb_flow_velocity": ([vp, vp], i32),
        "lb_flow_classes": ([vp, vp, P(i64), P(i64)], i32),
        "lb_flow_free": ([vp], None),
        "mp_workspace_bytes": ([P(vp), P(Species), i32, i32, i64, P(sz)], i32),
        "mp_init": ([P(vp), P(Species), i32, i32, i64, vp, sz, vp, P(vp)], i32),
        "mp_init_charged": ([P(vp), P(Species), P(vp), i32, i32, i64, vp, sz, vp, P(vp)], i32),
        "mp_step_n": ([vp, i64], i32),
        "mp_vacf": ([vp, i32, i64, i64, vp, vp, vp, vp], i32),
        "mp_uptake_init": ([P(vp), P(Species), i32, i32, i64, vp, sz, vp, P(vp)], i32),
        "mp_uptake": ([vp, i32, i64, i64, vp, vp], i32),
        "mp_steps_done": ([vp, P(i64)], i32),
        "mp_stats": ([vp, i32, P(Stats)], i32),
        "mp_state": ([vp, i32, i32, vp, vp], i32),
        "mp_profile_steps": ([vp, i64, P(dbl), P(dbl)], i32),
        "mp_checkpoint_bytes": ([vp, P(ctypes.c_size_t)], i32),
        "mp_save": ([vp, vp, ctypes.c_size_t], i32),
        "mp_load": ([vp, vp, ctypes.c_size_t], i32),
        "mp_free": ([vp], None),
        "sg_param_count": ([P(i64)], i32),
        "sg_workspace_bytes": ([i32, P(sz)], i32),
        "sg_create": ([i32, ctypes.c_uint64, vp, sz, vp, P(vp)], i32),
        "sg_set_params": ([vp, vp], i32),
        "sg_get_params": ([vp, vp], i32),
        "sg_set_normalization": ([vp, vp, vp, ctypes.c_float, ctypes.c_float], i32),
        "sg_train_step": ([vp, vp, vp, vp, i32, ctypes.c_float, vp], i32),
        "sg_gradients": ([vp, vp, vp, i32, vp, vp], i32),
        "sg_predict": ([vp, vp, i64, vp], i32),
        "sg_sync": ([vp], i32),
        "sg_free": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int):
    if status != LBMP_OK:
        raise LbmpError(status, _lib.lbmp_last_error().decode())


def _torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("liblbmp needs a ROCm GPU; none is visible")
    return torch


def _enter(stream, *tensors):
    """Order work queued on `stream` after the caller's current stream (which
    produced the tensors and the workspaces' previous contents), and tell the
    caching allocator that `stream` uses the tensors."""
    import torch
    stream.wait_stream(torch.cuda.current_stream())
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def _leave(stream):
    """Order the caller's current stream after the work just queued on `stream`
    (so results can be used there without an explicit synchronisation)."""
    import torch
    torch.cuda.current_stream().wait_stream(stream)


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _geometry(mask: np.ndarray, periodic=(1, 1, 1), iface_nbhd: int = 18):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if m.ndim != 3:
        raise ValueError("mask must be (nz, ny, nx)")
    nz, ny, nx = m.shape
    g = Geometry(nx, ny, nz, (ctypes.c_int * 3)(*periodic), ctypes.c_void_p(m.ctypes.data), iface_nbhd)
    return g, m


class Flow:
    """A flow handle and the device workspace it lives in."""

    def __init__(self, handle, ws, mask, geom, stream, steps=0, residual=0.0, converged=True):
        self.handle, self.ws, self.mask, self._geom, self.stream = handle, ws, mask, geom, stream
        self.steps, self.residual, self.converged = steps, residual, converged
        self.shape = mask.shape

    def velocity(self) -> np.ndarray:
        u = np.zeros((3,) + self.shape)
        _check(_lib.lb_flow_velocity(self.handle, _ptr(u)))
        return u

    def classes(self):
        cls = np.zeros(self.shape, dtype=np.int8)
        nf, ni = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.lb_flow_classes(self.handle, _ptr(cls), ctypes.byref(nf), ctypes.byref(ni)))
        return cls, nf.value, ni.value

    def free(self):
        if self.handle:
            _lib.lb_flow_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lb_flow_solve(mask, tau: float = 1.0, force=(0.0, 0.0, 0.0), tol: float = 1e-10,
                  max_steps: int = 200000, check_every: int = 100, periodic=(1, 1, 1),
                  iface_nbhd: int = 18, stream=None, allow_unconverged: bool = False) -> Flow:
    """Steady BGK flow (C-ABI lb_flow_solve). Returns a Flow."""
    torch = _torch_cuda()
    load_library()
    g, m = _geometry(mask, periodic, iface_nbhd)
    pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.lb_flow_workspace_bytes(ctypes.byref(g), ctypes.byref(pb), ctypes.byref(sb)))
    ws = torch.empty(pb.value, dtype=torch.uint8, device="cuda")
    scratch = torch.empty(sb.value, dtype=torch.uint8, device="cuda")
    stream = stream or torch.cuda.Stream()
    _enter(stream, ws, scratch)
    f = (ctypes.c_double * 3)(*force)
    h = ctypes.c_void_p()
    steps, res = ctypes.c_int64(), ctypes.c_double()
    st = _lib.lb_flow_solve(ctypes.byref(g), tau, f, tol, max_steps, check_every,
                            ctypes.c_void_p(ws.data_ptr()), pb.value,
                            ctypes.c_void_p(scratch.data_ptr()), sb.value,
                            ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h),
                            ctypes.byref(steps), ctypes.byref(res))
    del scratch
    if st == -4 and allow_unconverged:
        return Flow(h, ws, m, g, stream, steps.value, res.value, False)
    _check(st)
    return Flow(h, ws, m, g, stream, steps.value, res.value, True)


def lb_flow_solve_static(mask, tau: float = 1.0, force=(0.0, 0.0, 0.0), tol: float = 1e-10,
                         max_steps: int = 200000, check_every: int = 100, periodic=(1, 1, 1),
                         iface_nbhd: int = 18, stream=None, ws=None, allow_unconverged: bool = False) -> Flow:
    """lb_flow_solve without a scratch workspace (C-ABI lb_flow_solve_static):
    the solve's scratch is the library's static device array. `ws`, the
    persistent workspace (uint8 CUDA tensor of lb_flow_workspace_bytes), may
    be passed in so that the call itself allocates nothing."""
    torch = _torch_cuda()
    load_library()
    g, m = _geometry(mask, periodic, iface_nbhd)
    pb = ctypes.c_size_t()
    _check(_lib.lb_flow_workspace_bytes(ctypes.byref(g), ctypes.byref(pb), None))
    if ws is None:
        ws = torch.empty(pb.value, dtype=torch.uint8, device="cuda")
    stream = stream or torch.cuda.Stream()
    _enter(stream, ws)
    f = (ctypes.c_double * 3)(*force)
    h = ctypes.c_void_p()
    steps, res = ctypes.c_int64(), ctypes.c_double()
    st = _lib.lb_flow_solve_static(ctypes.byref(g), tau, f, tol, max_steps, check_every,
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h),
                                   ctypes.byref(steps), ctypes.byref(res))
    if st == -4 and allow_unconverged:
        return Flow(h, ws, m, g, stream, steps.value, res.value, False)
    _check(st)
    return Flow(h, ws, m, g, stream, steps.value, res.value, True)


def lb_flow_static_max_nodes() -> int:
    return int(load_library().lb_flow_static_max_nodes())


def lb_flow_from_velocity(mask, u, periodic=(1, 1, 1), iface_nbhd: int = 18, stream=None) -> Flow:
    """Flow handle from a given velocity field (3, nz, ny, nx)."""
    torch = _torch_cuda()
    load_library()
    g, m = _geometry(mask, periodic, iface_nbhd)
    ua = np.ascontiguousarray(u, dtype=np.float64)
    if ua.shape != (3,) + m.shape:
        raise ValueError("velocity must be (3, nz, ny, nx)")
    pb = ctypes.c_size_t()
    _check(_lib.lb_flow_workspace_bytes(ctypes.byref(g), ctypes.byref(pb), None))
    ws = torch.empty(pb.value, dtype=torch.uint8, device="cuda")
    stream = stream or torch.cuda.Stream()
    _enter(stream, ws)
    h = ctypes.c_void_p()
    _check(_lib.lb_flow_from_velocity(ctypes.byref(g), _ptr(ua), ctypes.c_void_p(ws.data_ptr()),
                                      pb.value, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
    return Flow(h, ws, m, g, stream)


def _species(sp: dict):
    ka = np.ascontiguousarray(np.atleast_1d(sp["k_a"]), dtype=np.float64)
    kd = np.ascontiguousarray(np.atleast_1d(sp["k_d"]), dtype=np.float64)
    if ka.shape != kd.shape:
        raise ValueError("k_a and k_d must have the same length")
    db = sp.get("D_b")
    dl = sp.get("Delta")
    s = Species(math.nan if db is None else float(db), math.nan if dl is None else float(dl),
                int(ka.size), ctypes.c_void_p(ka.ctypes.data), ctypes.c_void_p(kd.ctypes.data))
    return s, (ka, kd)


class MP:
    """A batched moment-propagation handle (C-ABI mp_*)."""

    def __init__(self, handle, ws, flows, n_species, stream, keep):
        self.handle, self.ws, self.flows, self.n_species, self.stream = handle, ws, flows, n_species, stream
        self._keep = keep

    def step(self, n: int):
        mp_step_n(self, n)

    def free(self):
        if self.handle:
            _lib.mp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def mp_init(flows, species, precision: int = LBMP_FP32, max_steps: int = 0, stream=None,
            _entry: str = "mp_init", beta_mu_ex=None) -> MP:
    """Set up moment propagation for flows[g] with species[g] = dict(D_b= or Delta=, k_a=, k_d=).
    beta_mu_ex: for charged tracers, one (nz, ny, nx) array (or None) per geometry
    (C-ABI mp_init_charged)."""
    torch = _torch_cuda()
    load_library()
    if isinstance(flows, Flow):
        flows = [flows]
    if isinstance(species, dict):
        species = [species]
    if len(flows) != len(species):
        raise ValueError("one species set per flow")
    n = len(flows)
    fl = (ctypes.c_void_p * n)(*[f.handle for f in flows])
    sps = (Species * n)()
    keep = []
    for i, sp in enumerate(species):
        s, k = _species(sp)
        sps[i] = s
        keep.append(k)
    nb = ctypes.c_size_t()
    _check(_lib.mp_workspace_bytes(fl, sps, n, precision, max_steps, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    stream = stream or torch.cuda.Stream()
    _enter(stream, ws)
    h = ctypes.c_void_p()
    if beta_mu_ex is not None:
        if isinstance(beta_mu_ex, np.ndarray):
            beta_mu_ex = [beta_mu_ex]
        if len(beta_mu_ex) != n:
            raise ValueError("one beta_mu_ex array (or None) per flow")
        arrs = []
        for f, b in zip(flows, beta_mu_ex):
            if b is None:
                arrs.append(None)
                continue
            a = np.ascontiguousarray(b, dtype=np.float64)
            if a.shape != f.shape:
                raise ValueError("beta_mu_ex must have the geometry's (nz, ny, nx) shape")
            arrs.append(a)
        keep.append(arrs)
        bp = (ctypes.c_void_p * n)(*[None if a is None else a.ctypes.data for a in arrs])
        _check(_lib.mp_init_charged(fl, sps, bp, n, precision, max_steps, ctypes.c_void_p(ws.data_ptr()),
                                    nb.value, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
    else:
        _check(getattr(_lib, _entry)(fl, sps, n, precision, max_steps, ctypes.c_void_p(ws.data_ptr()), nb.value,
                                     ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
    return MP(h, ws, list(flows), [int(s.n_species) for s in sps], stream, keep)


def mp_uptake_init(flows, species, precision: int = LBMP_FP32, max_steps: int = 0, stream=None) -> MP:
    """Out-of-equilibrium uptake: uniform mobile start, k_d = 0 allowed."""
    return mp_init(flows, species, precision, max_steps, stream, _entry="mp_uptake_init")


def mp_uptake(mp: MP, geom: int = 0, t0: int = 0, count: int | None = None) -> dict:
    """mobile, adsorbed (S, count) totals for tau = t0..t0+count-1."""
    S = mp.n_species[geom]
    if count is None:
        count = mp_steps_done(mp) - t0
    mob = np.zeros((S, count))
    ads = np.zeros((S, count))
    _check(_lib.mp_uptake(mp.handle, geom, t0, count, _ptr(mob), _ptr(ads)))
    return {"mobile": mob, "adsorbed": ads}


def mp_step_n(mp: MP, n: int):
    """Queue n steps on the handle's stream (asynchronous; ordered after the
    caller's current stream)."""
    _enter(mp.stream)
    _check(_lib.mp_step_n(mp.handle, int(n)))


def mp_profile_steps(mp: MP, n: int):
    """Run n steps with HIP events around each propagation-kernel launch.
    Returns (summed propagation-kernel ms, total ms)."""
    k, t = ctypes.c_double(), ctypes.c_double()
    _check(_lib.mp_profile_steps(mp.handle, int(n), ctypes.byref(k), ctypes.byref(t)))
    return k.value, t.value


def mp_steps_done(mp: MP) -> int:
    t = ctypes.c_int64()
    _check(_lib.mp_steps_done(mp.handle, ctypes.byref(t)))
    return t.value


def mp_vacf(mp: MP, geom: int = 0, t0: int = 0, count: int | None = None) -> dict:
    """Z (S, 3, count), D (S, 3, count), mass (S, 2), vbar (S, 3) for t = t0..t0+count-1."""
    S = mp.n_species[geom]
    if count is None:
        count = mp_steps_done(mp) + 1 - t0
    Z = np.zeros((S, 3, count))
    D = np.zeros((S, 3, count))
    mass = np.zeros((S, 2))
    vbar = np.zeros((S, 3))
    _check(_lib.mp_vacf(mp.handle, geom, t0, count, _ptr(Z), _ptr(D), _ptr(mass), _ptr(vbar)))
    return {"Z": Z, "D": D, "mass": mass, "vbar": vbar}


def mp_stats(mp: MP, geom: int = 0) -> dict:
    st = Stats()
    _check(_lib.mp_stats(mp.handle, geom, ctypes.byref(st)))
    return {"n_nodes": st.n_nodes, "n_fluid": st.n_fluid, "n_iface": st.n_iface,
            "lambda": st.lambda_, "min_p": st.min_p, "max_cell_peclet": st.max_cell_peclet,
            "min_stay": st.min_stay, "mean_velocity": list(st.mean_velocity),
            "tile_k": st.tile_k, "species_per_block": st.species_per_block,
            "kernel_variant": st.kernel_variant}


def mp_state(mp: MP, geom: int, species: int):
    """Current (X, Xads), each (4, nz, ny, nx) in FP64: density and x, y, z first moments."""
    shape = mp.flows[geom].shape
    X = np.zeros((4,) + shape)
    Xa = np.zeros((4,) + shape)
    _check(_lib.mp_state(mp.handle, geom, species, _ptr(X), _ptr(Xa)))
    return X, Xa


def mp_save(mp: MP) -> np.ndarray:
    """Checkpoint of the handle's current state (host bytes; see mp_load)."""
    n = ctypes.c_size_t()
    _check(_lib.mp_checkpoint_bytes(mp.handle, ctypes.byref(n)))
    buf = np.empty(n.value, dtype=np.uint8)
    _check(_lib.mp_save(mp.handle, _ptr(buf), buf.nbytes))
    return buf


def mp_load(mp: MP, buf) -> None:
    """Restores a checkpoint written by mp_save into a handle of the same workload."""
    b = np.ascontiguousarray(np.frombuffer(buf, dtype=np.uint8) if not isinstance(buf, np.ndarray) else buf)
    _check(_lib.mp_load(mp.handle, _ptr(b), b.nbytes))


def version() -> str:
    return load_library().lbmp_version().decode()


# ---------------------------------------------------------------- surrogate
class Surrogate:
    """BF16-MFMA MLP (C-ABI sg_*): features (porosity, specific surface, Pe,
    log10 k_a, log10 k_d, log10 t) -> log10(D_x(t)/D_b)."""

    def __init__(self, batch_max: int = 1024, seed: int = 0, stream=None):
        torch = _torch_cuda()
        load_library()
        nb = ctypes.c_size_t()
        _check(_lib.sg_workspace_bytes(batch_max, ctypes.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        self.stream = stream or torch.cuda.Stream()
        _enter(self.stream, self.ws)
        self.batch_max = batch_max
        h = ctypes.c_void_p()
        _check(_lib.sg_create(batch_max, seed, ctypes.c_void_p(self.ws.data_ptr()), nb.value,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int64()
        _check(_lib.sg_param_count(ctypes.byref(n)))
        self.n_params = n.value

    def set_params(self, p: np.ndarray):
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == self.n_params
        _check(_lib.sg_set_params(self.handle, _ptr(a)))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.n_params, dtype=np.float32)
        _check(_lib.sg_get_params(self.handle, _ptr(a)))
        return a

    def set_normalization(self, x_mean, x_std, y_mean: float, y_std: float):
        m = np.ascontiguousarray(x_mean, dtype=np.float32)
        s = np.ascontiguousarray(x_std, dtype=np.float32)
        _check(_lib.sg_set_normalization(self.handle, _ptr(m), _ptr(s), float(y_mean), float(y_std)))

    def train_step(self, x, y, idx, B: int, lr: float, want_loss: bool = False):
        """x, y: torch float32 CUDA tensors (n, 6), (n,); idx: int32 CUDA tensor (>= B) or None."""
        loss = ctypes.c_float()
        _enter(self.stream, x, y, idx)
        _check(_lib.sg_train_step(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                  ctypes.c_void_p(idx.data_ptr()) if idx is not None else None, int(B),
                                  float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def gradients(self, x, y, B: int):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_float()
        _enter(self.stream, x, y)
        _check(_lib.sg_gradients(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                 int(B), _ptr(g), ctypes.byref(loss)))
        return g, loss.value

    def predict(self, x, out=None):
        """x: torch float32 CUDA tensor (n, 6) -> torch float32 CUDA tensor (n,).
        Runs on the handle's stream after the caller's current stream's work;
        the current stream waits for the result."""
        torch = _torch_cuda()
        n = x.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device="cuda")
        _enter(self.stream, x, out)
        _check(_lib.sg_predict(self.handle, ctypes.c_void_p(x.data_ptr()), n, ctypes.c_void_p(out.data_ptr())))
        _leave(self.stream)
        return out

    def sync(self):
        _check(_lib.sg_sync(self.handle))

    def free(self):
        if self.handle:
            _lib.sg_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
