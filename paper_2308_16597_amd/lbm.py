"""Thin ctypes binding of include/lbm.h (argument marshalling only).

Every function of the C ABI is exposed under its own name; `Sim` bundles a
handle with numpy outputs.  PyTorch supplies device memory (an arena tensor)
and the HIP stream when it is importable and a GPU is present.

The library must have been built in-tree (paper_2308_16597_amd/libptlbm.so);
importing this module without it raises, there is no fallback path.
"""
import ctypes
import os
import re

import numpy as np

try:
    # torch ships its own HIP runtime (libamdhip64.so); loading torch first makes
    # the library bind to that same runtime instead of a second copy from
    # /opt/rocm, so that torch-allocated arenas and streams are valid here.
    import torch  # noqa: F401
except ImportError:
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libptlbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbm.h")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ESEED, LBM_EUNSTABLE, LBM_ESTATE, LBM_EBUDGET = \
    0, -1, -2, -3, -4, -5, -6, -7
STORE = {"f64": 0, "f32": 1, "shift_f32": 2, "shift_f16": 3, "shift_bf16": 4}
STREAMING = {"two_sets": 0, "in_place": 1}
LBM_LINKS_INDIRECT, LBM_LINKS_DIRECT = 0, 1
PHASES = ("links", "particles", "mask", "lattice", "refill", "collect")
STATS = ("steps", "links", "newborn", "ms_per_step", "gbps", "particles", "nodes", "bytes")

_d, _i = ctypes.c_double, ctypes.c_int32


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("abi_version", _i), ("nx", _i), ("ny", _i), ("periodic_x", _i), ("periodic_y", _i),
        ("storage", _i), ("rho0", _d), ("nu", _d), ("alpha", _d), ("gravity", _d), ("beta", _d),
        ("T_ref", _d), ("body_fx", _d), ("s_e", _d), ("s_eps", _d), ("s_q", _d), ("a_T", _d),
        ("sT_e", _d), ("sT_p", _d), ("wall_T", _d * 2), ("wall_ux", _d * 2), ("T_fluid0", _d),
        ("particle_T", _d), ("rho_ratio", _d), ("repulsion", _i), ("rep_eps", _d),
        ("rep_range", _d), ("T_shift", _d), ("max_particles", _i), ("max_diameter", _d),
        ("side_T", _d * 2), ("streaming", _i),
    ]


class LbmError(RuntimeError):
    def __init__(self, rc, msg):
        super().__init__(f"lbm error {rc}: {msg}")
        self.rc = rc


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2308_16597_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, P = ctypes.c_void_p, ctypes.POINTER
    L.lbm_abi_version.restype = _i
    L.lbm_params_default.argtypes = [P(LbmParams)]
    L.lbm_params_default.restype = None
    L.lbm_bytes_required.argtypes = [P(LbmParams)]
    L.lbm_bytes_required.restype = ctypes.c_size_t
    L.lbm_check_budget.argtypes = [P(LbmParams), ctypes.c_size_t]
    L.lbm_collect_lds_bytes.argtypes = [P(LbmParams)]
    L.lbm_collect_lds_bytes.restype = ctypes.c_size_t
    L.lbm_create.argtypes = [P(LbmParams), vp, P(vp)]
    L.lbm_create_in_arena.argtypes = [P(LbmParams), vp, ctypes.c_size_t, vp, P(vp)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_rsa_seed.argtypes = [_i, _i, _i, _d, _d, ctypes.c_uint64, vp]
    L.lbm_seed_particles.argtypes = [vp, _i, _d, _d, ctypes.c_uint64]
    L.lbm_set_particles.argtypes = [vp, _i, vp]
    L.lbm_set_particles_ellipse.argtypes = [vp, _i, vp]
    L.lbm_set_equilibrium.argtypes = [vp, vp, vp, vp, vp]
    L.lbm_step.argtypes = [vp, _i]
    L.lbm_set_addressing.argtypes = [vp, _i]
    L.lbm_step_many.argtypes = [vp, _i, vp, vp]
    L.lbm_step_many_noalloc.argtypes = [vp, _i, vp, vp]
    L.lbm_sync.argtypes = [vp]
    L.lbm_read_fields.argtypes = [vp, vp, vp, vp, vp, vp]
    L.lbm_read_particles.argtypes = [vp, vp, P(_i)]
    L.lbm_read_links.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, P(ctypes.c_int64)]
    L.lbm_time_phases.argtypes = [vp, _i, vp]
    L.lbm_stats.argtypes = [vp, vp]
    L.lbm_time_copy.argtypes = [vp, _i, vp]
    return L


_lib = _load()


def declared_functions():
    """Names of the functions include/lbm.h declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(lbm_\w+)\s*\(", text, re.M)))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, h=None):
    if rc != LBM_OK:
        raise LbmError(rc, _lib.lbm_last_error(h).decode())
    return rc


# --- the C ABI, one Python function per entry point -------------------------

def lbm_abi_version():
    return _lib.lbm_abi_version()


def lbm_params_default(**overrides):
    p = LbmParams()
    _lib.lbm_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if k in ("wall_T", "wall_ux", "side_T"):
            getattr(p, k)[0], getattr(p, k)[1] = float(v[0]), float(v[1])
        elif k == "storage" and isinstance(v, str):
            p.storage = STORE[v]
        elif k == "streaming" and isinstance(v, str):
            p.streaming = STREAMING[v]
        elif not hasattr(p, k):
            raise KeyError(k)
        else:
            setattr(p, k, v)
    return p


def lbm_bytes_required(p):
    return _lib.lbm_bytes_required(ctypes.byref(p))


def lbm_check_budget(p, budget_bytes):
    """LBM_OK if a run with these parameters fits budget_bytes of device
    memory, LBM_EBUDGET if not, LBM_EINVAL for invalid parameters."""
    return _lib.lbm_check_budget(ctypes.byref(p), int(budget_bytes))


def lbm_collect_lds_bytes(p):
    return _lib.lbm_collect_lds_bytes(ctypes.byref(p))


def lbm_create(p, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.lbm_create(ctypes.byref(p), stream, ctypes.byref(h)))
    return h


def lbm_create_in_arena(p, dev_ptr, nbytes, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.lbm_create_in_arena(ctypes.byref(p), ctypes.c_void_p(dev_ptr), nbytes, stream,
                                    ctypes.byref(h)))
    return h


def lbm_destroy(h):
    _lib.lbm_destroy(h)


def lbm_last_error(h=None):
    return _lib.lbm_last_error(h).decode()


def lbm_rsa_seed(nx, ny, n, diameter, min_gap, seed):
    out = np.zeros((max(n, 1), 7))
    _check(_lib.lbm_rsa_seed(nx, ny, n, diameter, min_gap, seed, _ptr(out)))
    return out[:n]


def lbm_seed_particles(h, n, diameter, min_gap, seed):
    _check(_lib.lbm_seed_particles(h, n, diameter, min_gap, seed), h)


def lbm_set_particles(h, rows7):
    rows7 = np.ascontiguousarray(rows7, dtype=np.float64).reshape(-1, 7)
    _check(_lib.lbm_set_particles(h, rows7.shape[0], _ptr(rows7)), h)


def lbm_set_particles_ellipse(h, rows8):
    rows8 = np.ascontiguousarray(rows8, dtype=np.float64).reshape(-1, 8)
    _check(_lib.lbm_set_particles_ellipse(h, rows8.shape[0], _ptr(rows8)), h)


def lbm_set_equilibrium(h, rho, ux, uy, T):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy, T)]
    _check(_lib.lbm_set_equilibrium(h, *[_ptr(a) for a in arrs]), h)


def lbm_set_addressing(h, mode):
    """mode: LBM_LINKS_INDIRECT or LBM_LINKS_DIRECT (or "indirect"/"direct")."""
    if isinstance(mode, str):
        mode = {"indirect": LBM_LINKS_INDIRECT, "direct": LBM_LINKS_DIRECT}[mode]
    _check(_lib.lbm_set_addressing(h, int(mode)), h)


def lbm_step(h, n):
    _check(_lib.lbm_step(h, int(n)), h)


def lbm_step_many(handles, nsteps, stream=None):
    """Advance handles[i] by nsteps[i] steps in batched launches."""
    n = len(handles)
    if n == 0:
        return
    hs = (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    ns = np.ascontiguousarray(nsteps, dtype=np.int32)
    if ns.shape != (n,):
        raise ValueError("one step count per handle")
    rc = _lib.lbm_step_many(ctypes.cast(hs, ctypes.c_void_p), n, _ptr(ns), stream)
    _check(rc, handles[0])


def lbm_step_many_noalloc(handles, nsteps, stream=None):
    """lbm_step_many from the library's fixed device array (allocates nothing)."""
    n = len(handles)
    if n == 0:
        return
    hs = (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    ns = np.ascontiguousarray(nsteps, dtype=np.int32)
    if ns.shape != (n,):
        raise ValueError("one step count per handle")
    rc = _lib.lbm_step_many_noalloc(ctypes.cast(hs, ctypes.c_void_p), n, _ptr(ns), stream)
    _check(rc, handles[0])


def lbm_sync(h):
    _check(_lib.lbm_sync(h), h)


def lbm_read_fields(h, nx, ny):
    rho, ux, uy, T = (np.empty((ny, nx)) for _ in range(4))
    owner = np.empty((ny, nx), dtype=np.int32)
    _check(_lib.lbm_read_fields(h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(owner)), h)
    return dict(rho=rho, ux=ux, uy=uy, T=T, owner=owner)


def lbm_read_particles(h):
    n = _i()
    _check(_lib.lbm_read_particles(h, None, ctypes.byref(n)), h)
    out = np.empty((n.value, 10))
    if n.value:
        _check(_lib.lbm_read_particles(h, _ptr(out), ctypes.byref(n)), h)
    return out


def lbm_read_links(h):
    n = ctypes.c_int64()
    _check(_lib.lbm_read_links(h, None, None, None, None, 0, ctypes.byref(n)), h)
    m = n.value
    node, d, part = (np.empty(m, dtype=np.int32) for _ in range(3))
    q = np.empty(m)
    if m:
        _check(_lib.lbm_read_links(h, _ptr(node), _ptr(d), _ptr(part), _ptr(q), m, ctypes.byref(n)), h)
    return dict(node=node, dir=d, particle=part, q=q)


def lbm_time_phases(h, nsteps):
    out = np.zeros(len(PHASES) + 3)
    _check(_lib.lbm_time_phases(h, int(nsteps), _ptr(out)), h)
    return dict(zip(PHASES + ("step", "lattice_overlapped", "step_overlapped"), out.tolist()))


def lbm_stats(h):
    out = np.zeros(len(STATS))
    _check(_lib.lbm_stats(h, _ptr(out)), h)
    d = dict(zip(STATS, out.tolist()))
    for k in ("steps", "links", "newborn", "particles", "nodes", "bytes"):
        d[k] = int(d[k])
    return d


def lbm_time_copy(h, reps):
    """Mean device ms of a plain copy of the run's 14 population arrays."""
    out = np.zeros(1)
    _check(_lib.lbm_time_copy(h, int(reps), _ptr(out)), h)
    return float(out[0])


# --- convenience wrapper -----------------------------------------------------

def step_many(sims, nsteps, stream=None):
    """Advance sims[i] by nsteps[i] steps together (batched launches)."""
    lbm_step_many([s.handle for s in sims], nsteps, stream)


class Sim:
    """One simulation on the GPU.

    With `torch_memory=True` (default) the device arena is a torch tensor and
    the work goes on torch's current HIP stream; otherwise the library
    allocates with hipMalloc and creates its own stream.
    """

    def __init__(self, params=None, torch_memory=True, arena=None, stream=None, **overrides):
        self.params = params if params is not None else lbm_params_default(**overrides)
        if params is not None and overrides:
            for k, v in overrides.items():
                setattr(self.params, k, v)
        self.nx, self.ny = self.params.nx, self.params.ny
        self._arena = None
        self._h = None
        if arena is not None:
            # a caller-owned slice (device pointer, bytes) of a larger buffer
            self._h = lbm_create_in_arena(self.params, int(arena[0]), int(arena[1]),
                                          ctypes.c_void_p(stream) if stream else None)
        elif torch_memory:
            import torch
            nbytes = lbm_bytes_required(self.params)
            if nbytes == 0:
                self._h = lbm_create(self.params)  # invalid parameters: raises with the reason
                return
            self._arena = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            stream = torch.cuda.current_stream().cuda_stream or None
            self._h = lbm_create_in_arena(self.params, self._arena.data_ptr(), nbytes,
                                          ctypes.c_void_p(stream) if stream else None)
        else:
            self._h = lbm_create(self.params)

    def close(self):
        if self._h:
            lbm_destroy(self._h)
            self._h = None
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def seed_particles(self, n, diameter, min_gap=1.0, seed=1):
        lbm_seed_particles(self._h, n, diameter, min_gap, seed)

    def set_particles(self, rows7):
        lbm_set_particles(self._h, rows7)

    def set_particles_ellipse(self, rows8):
        lbm_set_particles_ellipse(self._h, rows8)

    def set_equilibrium(self, rho, ux, uy, T):
        lbm_set_equilibrium(self._h, rho, ux, uy, T)

    def step(self, n=1):
        lbm_step(self._h, n)

    def set_addressing(self, mode):
        lbm_set_addressing(self._h, mode)

    @property
    def handle(self):
        return self._h

    def sync(self):
        lbm_sync(self._h)

    def fields(self):
        return lbm_read_fields(self._h, self.nx, self.ny)

    def particles(self):
        return lbm_read_particles(self._h)

    def links(self):
        return lbm_read_links(self._h)

    def time_phases(self, nsteps):
        return lbm_time_phases(self._h, nsteps)

    def stats(self):
        return lbm_stats(self._h)

    def time_copy(self, reps=10):
        return lbm_time_copy(self._h, reps)
