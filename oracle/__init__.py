"""ctypes binding of the CPU oracle (test infrastructure only).

The oracle is a plain single-threaded FP64 C implementation of the
particle-resolved thermal lattice Boltzmann method of Xu & Li (arXiv
2308.16597).  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the GPU library never does.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

_c_d = ctypes.c_double
_c_i = ctypes.c_int32
_P = np.ctypeslib.ndpointer


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", _c_i), ("ny", _c_i), ("periodic_x", _c_i), ("periodic_y", _c_i),
        ("rho0", _c_d), ("nu", _c_d), ("alpha", _c_d),
        ("gravity", _c_d), ("beta", _c_d), ("T_ref", _c_d), ("body_fx", _c_d),
        ("s_e", _c_d), ("s_eps", _c_d), ("s_q", _c_d),
        ("a_T", _c_d), ("sT_e", _c_d), ("sT_p", _c_d),
        ("wall_T", _c_d * 2), ("wall_ux", _c_d * 2),
        ("T_fluid0", _c_d), ("particle_T", _c_d), ("rho_ratio", _c_d),
        ("repulsion", _c_i), ("rep_eps", _c_d), ("rep_range", _c_d),
        ("side_T", _c_d * 2),
    ]


DEFAULTS = dict(nx=32, ny=32, periodic_x=1, periodic_y=0, rho0=1.0, nu=0.1, alpha=0.1,
                gravity=0.0, beta=0.0, T_ref=0.0, body_fx=0.0, s_e=0.0, s_eps=0.0,
                s_q=0.0, a_T=-2.0, sT_e=0.0, sT_p=0.0, wall_T=(0.0, 0.0),
                wall_ux=(0.0, 0.0), T_fluid0=0.0, particle_T=1.0, rho_ratio=1.5,
                repulsion=1, rep_eps=1e-3, rep_range=3.0, side_T=(0.0, 0.0))


def make_params(**kw):
    d = dict(DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise KeyError(f"unknown oracle parameters: {sorted(unknown)}")
    d.update(kw)
    p = OrcParams()
    for k, v in d.items():
        if k in ("wall_T", "wall_ux", "side_T"):
            getattr(p, k)[0], getattr(p, k)[1] = float(v[0]), float(v[1])
        else:
            setattr(p, k, v)
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        vp = ctypes.c_void_p
        dp = ctypes.POINTER(_c_d)
        L.orc_create.argtypes = [ctypes.POINTER(OrcParams), ctypes.POINTER(vp)]
        L.orc_destroy.argtypes = [vp]
        L.orc_last_error.argtypes = [vp]
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_set_particles.argtypes = [vp, _c_i, vp]
        L.orc_set_particles_ellipse.argtypes = [vp, _c_i, vp]
        L.orc_link_q_ellipse.argtypes = [_c_d, _c_d, _c_d, _c_d, _c_d, _c_i]
        L.orc_link_q_ellipse.restype = _c_d
        L.orc_inside_shape.argtypes = [_c_d, _c_d, _c_d, _c_d, _c_d]
        L.orc_inside_shape.restype = _c_i
        L.orc_refill_direction.argtypes = [_c_d, _c_d, _c_d, _c_d, _c_d]
        L.orc_refill_direction.restype = _c_i
        L.orc_repulsion_pair_ellipse.argtypes = [ctypes.POINTER(OrcParams)] + [_c_d] * 10 + [vp]
        L.orc_repulsion_walls_ellipse.argtypes = [ctypes.POINTER(OrcParams)] + [_c_d] * 5 + [vp]
        L.orc_newton_euler_ellipse.argtypes = [ctypes.POINTER(OrcParams), vp, _c_d, _c_d, _c_d,
                                               _c_d, vp]
        L.orc_set_equilibrium.argtypes = [vp, vp, vp, vp, vp]
        L.orc_step.argtypes = [vp, _c_i]
        L.orc_steps_done.argtypes = [vp]
        L.orc_steps_done.restype = ctypes.c_int64
        L.orc_read_fields.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_read_populations.argtypes = [vp, vp, vp]
        L.orc_read_particles.argtypes = [vp, vp, ctypes.POINTER(_c_i)]
        L.orc_read_links.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64)]
        L.orc_nusselt.argtypes = [vp, dp, dp]
        L.orc_collide_node.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_link_q.argtypes = [_c_d, _c_d, _c_d, _c_i]
        L.orc_link_q.restype = _c_d
        L.orc_bouzidi.argtypes = [_c_d, _c_i, _c_d, _c_d, _c_d, _c_d, _c_d, _c_i, _c_i,
                                  _c_d, _c_d, _c_d]
        L.orc_bouzidi.restype = _c_d
        L.orc_thermal_link.argtypes = [_c_d, _c_i, _c_d, _c_d, _c_d, _c_i, _c_d, _c_d]
        L.orc_thermal_link.restype = _c_d
        L.orc_repulsion_pair.argtypes = [ctypes.POINTER(OrcParams), _c_d, _c_d, _c_d,
                                         _c_d, _c_d, _c_d, vp]
        L.orc_repulsion_walls.argtypes = [ctypes.POINTER(OrcParams), _c_d, _c_d, _c_d, vp]
        L.orc_newton_euler.argtypes = [ctypes.POINTER(OrcParams), vp, _c_d, _c_d, _c_d, vp]
        L.orc_refill_node.argtypes = [vp, _c_i, vp, vp, vp, _c_d, _c_d, vp, vp]
        L.orc_rates.argtypes = [vp, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, rc, msg):
        super().__init__(f"oracle error {rc}: {msg}")
        self.rc = rc


class Oracle:
    """One oracle run.  Parameters are the fields of OrcParams."""

    def __init__(self, **params):
        self.params = make_params(**params)
        self.nx, self.ny = self.params.nx, self.params.ny
        h = ctypes.c_void_p()
        rc = lib().orc_create(ctypes.byref(self.params), ctypes.byref(h))
        self._h = h
        if rc != 0:
            msg = lib().orc_last_error(h).decode() if h else ""
            if h:
                lib().orc_destroy(h)
            self._h = None
            raise OracleError(rc, msg)

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != 0:
            raise OracleError(rc, lib().orc_last_error(self._h).decode())

    def set_particles(self, rows7):
        rows7 = np.ascontiguousarray(rows7, dtype=np.float64).reshape(-1, 7)
        self._check(lib().orc_set_particles(self._h, rows7.shape[0], _ptr(rows7)))

    def set_particles_ellipse(self, rows8):
        rows8 = np.ascontiguousarray(rows8, dtype=np.float64).reshape(-1, 8)
        self._check(lib().orc_set_particles_ellipse(self._h, rows8.shape[0], _ptr(rows8)))

    def set_equilibrium(self, rho, ux, uy, T):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny, self.nx)
                for a in (rho, ux, uy, T)]
        self._check(lib().orc_set_equilibrium(self._h, *[_ptr(a) for a in arrs]))

    def step(self, n=1):
        self._check(lib().orc_step(self._h, int(n)))

    @property
    def steps_done(self):
        return lib().orc_steps_done(self._h)

    def fields(self):
        shp = (self.ny, self.nx)
        rho, ux, uy, T = (np.empty(shp) for _ in range(4))
        owner = np.empty(shp, dtype=np.int32)
        self._check(lib().orc_read_fields(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T),
                                          _ptr(owner)))
        return dict(rho=rho, ux=ux, uy=uy, T=T, owner=owner)

    def populations(self):
        f = np.empty((9, self.ny, self.nx))
        g = np.empty((5, self.ny, self.nx))
        self._check(lib().orc_read_populations(self._h, _ptr(f), _ptr(g)))
        return f, g

    def particles(self):
        n = _c_i()
        lib().orc_read_particles(self._h, None, ctypes.byref(n))
        out = np.empty((n.value, 10))
        self._check(lib().orc_read_particles(self._h, _ptr(out), ctypes.byref(n)))
        return out

    def links(self):
        n = ctypes.c_int64()
        self._check(lib().orc_read_links(self._h, None, None, None, None, 0, ctypes.byref(n)))
        m = n.value
        node = np.empty(m, dtype=np.int32)
        d = np.empty(m, dtype=np.int32)
        part = np.empty(m, dtype=np.int32)
        q = np.empty(m)
        self._check(lib().orc_read_links(self._h, _ptr(node), _ptr(d), _ptr(part), _ptr(q), m,
                                         ctypes.byref(n)))
        return dict(node=node, dir=d, particle=part, q=q)

    def nusselt(self):
        a, b = _c_d(), _c_d()
        self._check(lib().orc_nusselt(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def rates(self):
        s9, s5, w5 = np.empty(9), np.empty(5), np.empty(5)
        lib().orc_rates(self._h, _ptr(s9), _ptr(s5), _ptr(w5))
        return s9, s5, w5

    def collide_node(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        fo, go, m = np.empty(9), np.empty(5), np.empty(4)
        lib().orc_collide_node(self._h, _ptr(f), _ptr(g), _ptr(fo), _ptr(go), _ptr(m))
        return fo, go, m

    def refill_node(self, K, f1, f2, f3, uwx, uwy):
        f1, f2, f3 = (np.ascontiguousarray(a, dtype=np.float64) for a in (f1, f2, f3))
        fo, go = np.empty(9), np.empty(5)
        lib().orc_refill_node(self._h, int(K), _ptr(f1), _ptr(f2), _ptr(f3), float(uwx),
                              float(uwy), _ptr(fo), _ptr(go))
        return fo, go


def link_q(dx, dy, r, i):
    return lib().orc_link_q(float(dx), float(dy), float(r), int(i))


def link_q_ellipse(dx, dy, a, b, theta, i):
    return lib().orc_link_q_ellipse(float(dx), float(dy), float(a), float(b), float(theta), int(i))


def inside_shape(dx, dy, a, b, theta):
    return bool(lib().orc_inside_shape(float(dx), float(dy), float(a), float(b), float(theta)))


def refill_direction(dx, dy, a, b, theta):
    return lib().orc_refill_direction(float(dx), float(dy), float(a), float(b), float(theta))


def bouzidi(q, i, fi_xf, fi_xf1, fi_xf2, fib_xf, fib_xf1, have1, have2, rho0, uwx, uwy):
    return lib().orc_bouzidi(q, i, fi_xf, fi_xf1, fi_xf2, fib_xf, fib_xf1, int(have1),
                             int(have2), rho0, uwx, uwy)


def thermal_link(q, i, gi_xf, gi_xf1, gib_xf, have1, w5_i, Tw):
    return lib().orc_thermal_link(q, i, gi_xf, gi_xf1, gib_xf, int(have1), w5_i, Tw)


def repulsion_pair(params, xp, yp, rp, xq, yq, rq):
    out = np.empty(2)
    lib().orc_repulsion_pair(ctypes.byref(params), xp, yp, rp, xq, yq, rq, _ptr(out))
    return out


def repulsion_walls(params, xp, yp, rp):
    out = np.empty(2)
    lib().orc_repulsion_walls(ctypes.byref(params), xp, yp, rp, _ptr(out))
    return out


def repulsion_pair_ellipse(params, p, q):
    """p, q: (x, y, a, b, theta) of the two particles."""
    out = np.empty(2)
    lib().orc_repulsion_pair_ellipse(ctypes.byref(params), *[float(v) for v in p],
                                     *[float(v) for v in q], _ptr(out))
    return out


def repulsion_walls_ellipse(params, x, y, a, b, theta):
    out = np.empty(2)
    lib().orc_repulsion_walls_ellipse(ctypes.byref(params), float(x), float(y), float(a), float(b),
                                      float(theta), _ptr(out))
    return out


def newton_euler_ellipse(params, state7, b, Fx, Fy, Tz):
    st = np.ascontiguousarray(state7, dtype=np.float64)
    out = np.empty(7)
    lib().orc_newton_euler_ellipse(ctypes.byref(params), _ptr(st), float(b), Fx, Fy, Tz, _ptr(out))
    return out


def newton_euler(params, state7, Fx, Fy, Tz):
    st = np.ascontiguousarray(state7, dtype=np.float64)
    out = np.empty(7)
    lib().orc_newton_euler(ctypes.byref(params), _ptr(st), Fx, Fy, Tz, _ptr(out))
    return out
