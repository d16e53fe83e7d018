"""ctypes wrapper of the plain FP64 CPU oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use it; the product path never does.  It
takes plain dicts describing the problem (see the workload descriptions) and
imports nothing from the GPU package.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

FAM = {"paper": 0, "cfg": 1}
SIGMA = {"poly": 0, "vhs": 1}


class OrcProblem(C.Structure):
    _fields_ = [
        ("family", C.c_int), ("L", C.c_double * 3), ("nphys", C.c_double),
        ("q", C.c_double), ("m", C.c_double), ("eps0", C.c_double), ("T", C.c_double),
        ("vbar", C.c_double), ("phibar", C.c_double), ("rho_amp", C.c_double),
        ("sigma_model", C.c_int), ("n_sigma", C.c_int), ("sigma_n", C.c_double * 3),
        ("sigma_ref", C.c_double), ("g_ref", C.c_double), ("omega", C.c_double),
        ("g_max", C.c_double), ("chi_model", C.c_int), ("field_to_particles", C.c_int),
        ("particles_to_field", C.c_int), ("collisions", C.c_int), ("isolate", C.c_int),
        ("coding_error", C.c_int), ("chi_alpha", C.c_double),
    ]


class OrcDisc(C.Structure):
    _fields_ = [("nc", C.c_int * 3), ("np", C.c_int64), ("dt", C.c_double), ("navg", C.c_int),
                ("cg_tol", C.c_double), ("cg_max_iter", C.c_int), ("poisson_op", C.c_int)]


class OrcPair(C.Structure):
    _fields_ = [("cell", C.c_int64), ("call", C.c_int64), ("k", C.c_int64), ("m", C.c_int64),
                ("p", C.c_int64), ("q", C.c_int64), ("accepted", C.c_int64),
                ("u_acc", C.c_double), ("ratio", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa: F401  (module import only)
            _b.build()
        L = C.CDLL(LIB_PATH)
        d, i64, u64, i32, vp = C.c_double, C.c_int64, C.c_uint64, C.c_int32, C.c_void_p
        P = C.POINTER
        L.orc_philox4x64_10.argtypes = [P(u64), P(u64), P(u64)]
        L.orc_u01.argtypes = [u64]; L.orc_u01.restype = d
        L.orc_u01_open.argtypes = [u64]; L.orc_u01_open.restype = d
        L.orc_index_below.argtypes = [u64, i64]; L.orc_index_below.restype = i64
        L.orc_init_uniforms.argtypes = [u64, C.c_uint32, i64, P(d)]
        for f in ("orc_xM", "orc_vM", "orc_vdotM"):
            getattr(L, f).argtypes = [P(OrcProblem), P(d), d, P(d)]
        L.orc_xdotM.argtypes = [P(OrcProblem), P(d), d, P(d)]
        for f in ("orc_fx", "orc_phiM", "orc_lapphiM"):
            getattr(L, f).argtypes = [P(OrcProblem), P(d), d]
            getattr(L, f).restype = d
        L.orc_EM.argtypes = [P(OrcProblem), P(d), d, P(d)]
        L.orc_vhat.argtypes = [P(OrcProblem), d, P(d)]
        L.orc_sigma_g.argtypes = [P(OrcProblem), d]; L.orc_sigma_g.restype = d
        L.orc_sigma_g_max.argtypes = [P(OrcProblem)]; L.orc_sigma_g_max.restype = d
        L.orc_source_integral.argtypes = [P(OrcProblem), P(d), d, P(d)]
        L.orc_hs_K.argtypes = [d]; L.orc_hs_K.restype = d
        L.orc_deposit.argtypes = [P(OrcProblem), P(OrcDisc), i64, P(d), P(d)]
        L.orc_rhs.argtypes = [P(OrcProblem), P(OrcDisc), P(d), d, P(d)]
        L.orc_cg.argtypes = [P(OrcDisc), P(OrcProblem), P(d), P(d), d, C.c_int, P(C.c_int), P(d)]
        L.orc_angle_record_start.argtypes = [P(d), C.c_int64]
        L.orc_angle_record_stop.argtypes = []
        L.orc_angle_record_stop.restype = C.c_int64
        L.orc_angle_errors.argtypes = [P(d), C.c_int64, C.c_int, d, P(d)]
        L.orc_cos_chi.argtypes = [C.c_int, d, d]
        L.orc_cos_chi.restype = d
        L.orc_chi_cdf.argtypes = [C.c_int, d, d]
        L.orc_chi_cdf.restype = d
        L.orc_laplacian.argtypes = [P(OrcDisc), P(OrcProblem), P(d), P(d)]
        L.orc_gradient.argtypes = [P(OrcProblem), P(OrcDisc), P(d), P(d)]
        L.orc_gather.argtypes = [P(OrcProblem), P(OrcDisc), P(d), i64, P(d), P(d)]
        L.orc_cell_keys.argtypes = [P(OrcProblem), P(OrcDisc), i64, P(d), P(i32)]
        L.orc_stable_sort.argtypes = [i64, i32, P(i32), P(i64), P(i64)]
        L.orc_collide_cell.argtypes = [P(OrcProblem), P(OrcDisc), u64, C.c_uint32, i64, C.c_int,
                                       i64, i64, P(d), P(d), P(OrcPair), i64, P(i64), P(i64),
                                       P(i64)]
        L.orc_create.argtypes = [P(OrcProblem), P(OrcDisc), u64, C.c_uint32]
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_init.argtypes = [vp]
        L.orc_step.argtypes = [vp, C.c_int]
        L.orc_collide.argtypes = [vp, C.c_int, d, P(d), P(d), P(OrcPair), i64, P(i64)]
        L.orc_errors.argtypes = [vp, P(d)]
        L.orc_get.argtypes = [vp, C.c_int, vp]
        L.orc_set.argtypes = [vp, C.c_int, vp]
        L.orc_step_index.argtypes = [vp]; L.orc_step_index.restype = i64
        L.orc_time.argtypes = [vp]; L.orc_time.restype = d
        L.orc_cg_iters.argtypes = [vp]
        L.orc_cg_relres.argtypes = [vp]; L.orc_cg_relres.restype = d
        L.orc_accepted.argtypes = [vp]; L.orc_accepted.restype = i64
        L.orc_gmax_events.argtypes = [vp]; L.orc_gmax_events.restype = i64
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_max_threads.argtypes = []
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_problem(p: dict) -> OrcProblem:
    s = OrcProblem()
    s.family = FAM[p["family"]]
    s.L = (C.c_double * 3)(*p["L"])
    for k in ("nphys", "q", "m", "eps0", "T", "vbar", "phibar", "rho_amp", "sigma_ref", "g_ref",
              "omega", "g_max"):
        setattr(s, k, float(p[k]))
    s.sigma_model = SIGMA[p["sigma_model"]]
    sn = list(p["sigma_n"]) + [0.0] * (3 - len(p["sigma_n"]))
    s.n_sigma = len(p["sigma_n"])
    s.sigma_n = (C.c_double * 3)(*sn)
    s.chi_model = int(p.get("chi_model", 0))
    s.chi_alpha = float(p.get("chi_alpha", 1.0))
    for k in ("field_to_particles", "particles_to_field", "collisions", "isolate"):
        setattr(s, k, int(p[k]))
    s.coding_error = int(p.get("coding_error", 0))
    return s


def make_disc(d: dict) -> OrcDisc:
    s = OrcDisc()
    s.nc = (C.c_int * 3)(*d["nc"])
    s.np = int(d["np"])
    s.dt = float(d["dt"])
    s.navg = int(d["navg"])
    s.cg_tol = float(d["cg_tol"])
    s.cg_max_iter = int(d["cg_max_iter"])
    s.poisson_op = int(d.get("poisson_op", 0))
    return s


# ---------------------------------------------------------------- pure functions
def philox_block(ctr, key):
    c = (C.c_uint64 * 4)(*[int(x) & (2**64 - 1) for x in ctr])
    k = (C.c_uint64 * 2)(*[int(x) & (2**64 - 1) for x in key])
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return [int(x) for x in o]


def set_threads(n: int) -> None:
    """Threads of the oracle's independent loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return lib().orc_max_threads()


def init_uniforms(seed, rep, pid):
    o = (C.c_double * 6)()
    lib().orc_init_uniforms(seed, rep, pid, o)
    return np.array(list(o))


def _vec3(fn, prob, a, t):
    P = make_problem(prob)
    i = (C.c_double * 3)(*a)
    o = (C.c_double * 3)()
    fn(C.byref(P), i, float(t), o)
    return np.array(list(o))


def xM(prob, xi3, t):
    return _vec3(lib().orc_xM, prob, xi3, t)


def vM(prob, xi3, t):
    return _vec3(lib().orc_vM, prob, xi3, t)


def xdotM(prob, xm3, t):
    return _vec3(lib().orc_xdotM, prob, xm3, t)


def vdotM(prob, xi3, t):
    return _vec3(lib().orc_vdotM, prob, xi3, t)


def EM(prob, x3, t):
    return _vec3(lib().orc_EM, prob, x3, t)


def source_integral(prob, v3, t):
    P = make_problem(prob)
    i = (C.c_double * 3)(*v3)
    o = (C.c_double * 3)()
    st = lib().orc_source_integral(C.byref(P), i, float(t), o)
    if st != 0:
        raise ValueError("no closed-form source for this cross section / family")
    return np.array(list(o))


def scalar(name, prob, x3, t):
    P = make_problem(prob)
    return getattr(lib(), name)(C.byref(P), (C.c_double * 3)(*x3), float(t))


def vhat(prob, t):
    P = make_problem(prob)
    o = (C.c_double * 3)()
    lib().orc_vhat(C.byref(P), float(t), o)
    return np.array(list(o))


def sigma_g(prob, g):
    P = make_problem(prob)
    return lib().orc_sigma_g(C.byref(P), float(g))


def sigma_g_max(prob):
    P = make_problem(prob)
    return lib().orc_sigma_g_max(C.byref(P))


def hs_K(lam):
    return lib().orc_hs_K(float(lam))


def deposit(prob, disc, x):
    """x: (3, np) positions in [0, L)."""
    P, D = make_problem(prob), make_disc(disc)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = int(np.prod(disc["nc"]))
    rho = np.zeros(n)
    lib().orc_deposit(C.byref(P), C.byref(D), x.shape[1], _dp(x), _dp(rho))
    return rho


def rhs(prob, disc, rho, t):
    P, D = make_problem(prob), make_disc(disc)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    b = np.zeros_like(rho)
    lib().orc_rhs(C.byref(P), C.byref(D), _dp(rho), float(t), _dp(b))
    return b


def cg(prob, disc, b, phi0=None, tol=None, max_iter=None):
    P, D = make_problem(prob), make_disc(disc)
    b = np.ascontiguousarray(b, dtype=np.float64)
    phi = np.zeros_like(b) if phi0 is None else np.array(phi0, dtype=np.float64)
    it = C.c_int()
    rr = C.c_double()
    st = lib().orc_cg(C.byref(D), C.byref(P), _dp(b), _dp(phi),
                      float(disc["cg_tol"] if tol is None else tol),
                      int(disc["cg_max_iter"] if max_iter is None else max_iter),
                      C.byref(it), C.byref(rr))
    return phi, it.value, rr.value, st


def laplacian(prob, disc, phi):
    P, D = make_problem(prob), make_disc(disc)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros_like(phi)
    lib().orc_laplacian(C.byref(D), C.byref(P), _dp(phi), _dp(out))
    return out


def gradient(prob, disc, phi):
    P, D = make_problem(prob), make_disc(disc)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    E = np.zeros(3 * phi.size)
    lib().orc_gradient(C.byref(P), C.byref(D), _dp(phi), _dp(E))
    return E.reshape(3, -1)


def gather(prob, disc, E, x):
    P, D = make_problem(prob), make_disc(disc)
    E = np.ascontiguousarray(E, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    Ep = np.zeros_like(x)
    lib().orc_gather(C.byref(P), C.byref(D), _dp(E), x.shape[1], _dp(x), _dp(Ep))
    return Ep


def cell_keys(prob, disc, x):
    P, D = make_problem(prob), make_disc(disc)
    x = np.ascontiguousarray(x, dtype=np.float64)
    k = np.zeros(x.shape[1], dtype=np.int32)
    lib().orc_cell_keys(C.byref(P), C.byref(D), x.shape[1], _dp(x),
                        k.ctypes.data_as(C.POINTER(C.c_int32)))
    return k


def stable_sort(keys, ncell):
    keys = np.ascontiguousarray(keys, dtype=np.int32)
    perm = np.zeros(keys.size, dtype=np.int64)
    cs = np.zeros(ncell + 1, dtype=np.int64)
    lib().orc_stable_sort(keys.size, ncell, keys.ctypes.data_as(C.POINTER(C.c_int32)),
                          perm.ctypes.data_as(C.POINTER(C.c_int64)),
                          cs.ctypes.data_as(C.POINTER(C.c_int64)))
    return perm, cs


def collide_cell(prob, disc, seed, rep, step, call, cell, v, log_cap=0):
    """v: (3, n) velocities of one cell.  Returns (dv_avg (3, n), pairs, n_acc, n_gmax)."""
    P, D = make_problem(prob), make_disc(disc)
    v = np.ascontiguousarray(v, dtype=np.float64)
    n = v.shape[1]
    dv = np.zeros_like(v)
    log = (OrcPair * max(1, log_cap))()
    ln, na, ng = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    lib().orc_collide_cell(C.byref(P), C.byref(D), seed, rep, step, call, cell, n, _dp(v), _dp(dv),
                           log if log_cap else None, log_cap, C.byref(ln), C.byref(na),
                           C.byref(ng))
    pairs = [(r.cell, r.call, r.k, r.m, r.p, r.q, r.accepted)
             for r in list(log)[:min(ln.value, log_cap)]] if log_cap else []
    return dv, pairs, na.value, ng.value


# ---------------------------------------------------------------- simulation
class Sim:
    """One manufactured-solution simulation run by the oracle."""

    X, V, ID, CELL_START, RHO, PHI, E, EP = range(8)

    def __init__(self, prob: dict, disc: dict, seed: int = 1, replicate: int = 0):
        self.prob, self.disc = prob, disc
        self._P, self._D = make_problem(prob), make_disc(disc)
        self.np = int(disc["np"])
        self.nn = int(np.prod(disc["nc"]))
        self.h = lib().orc_create(C.byref(self._P), C.byref(self._D), seed, replicate)

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the process releases the memory anyway
        if getattr(self, "h", None) and not _finalizing():
            lib().orc_destroy(self.h)
            self.h = None

    def init(self):
        return lib().orc_init(self.h)

    def step(self, n=1):
        return lib().orc_step(self.h, n)

    def get(self, what):
        if what in (self.X, self.V, self.EP):
            a = np.zeros((3, self.np))
        elif what == self.ID:
            a = np.zeros(self.np, dtype=np.int64)
        elif what == self.CELL_START:
            a = np.zeros(self.nn + 1, dtype=np.int64)
        elif what == self.E:
            a = np.zeros((3, self.nn))
        else:
            a = np.zeros(self.nn)
        lib().orc_get(self.h, what, a.ctypes.data)
        return a

    def set(self, what, a):
        a = np.ascontiguousarray(a)
        return lib().orc_set(self.h, what, a.ctypes.data)

    def collide(self, call, t, log_cap=0):
        dv = np.zeros((3, self.np))
        src = np.zeros((3, self.np))
        log = (OrcPair * max(1, log_cap))()
        ln = C.c_int64(0)
        st = lib().orc_collide(self.h, call, float(t), _dp(dv), _dp(src),
                               log if log_cap else None, log_cap, C.byref(ln))
        recs = list(log)[:min(ln.value, log_cap)] if log_cap else []
        pairs = [(r.cell, r.call, r.k, r.m, r.p, r.q, r.accepted) for r in recs]
        # the accept test's two sides per logged pair: (U, sigma g / (sigma g)_max)
        self.last_accept_test = np.array([(r.u_acc, r.ratio) for r in recs]).reshape(-1, 2)
        return dv, src, pairs, ln.value, st

    def errors(self):
        o = (C.c_double * 14)()
        lib().orc_errors(self.h, o)
        o = list(o)
        return {"l2": np.array(o[:7]), "linf": np.array(o[7:])}

    @property
    def step_index(self):
        return lib().orc_step_index(self.h)

    @property
    def time(self):
        return lib().orc_time(self.h)

    @property
    def cg_iters(self):
        return lib().orc_cg_iters(self.h)

    @property
    def cg_relres(self):
        return lib().orc_cg_relres(self.h)

    @property
    def accepted(self):
        return lib().orc_accepted(self.h)

    @property
    def gmax_events(self):
        return lib().orc_gmax_events(self.h)


class AngleRecorder:
    """Collects (chi, eps) of every accepted oracle collision inside a with-block
    (eq. angle_recovery); .records is an [n, 2] array afterwards."""

    def __init__(self, capacity=1 << 22):
        self.buf = np.zeros(2 * capacity)
        self.capacity = capacity
        self.records = None
        self.total = 0

    def __enter__(self):
        lib().orc_angle_record_start(_dp(self.buf), self.capacity)
        return self

    def __exit__(self, *exc):
        self.total = lib().orc_angle_record_stop()
        n = min(self.total, self.capacity)
        self.records = self.buf[: 2 * n].reshape(n, 2).copy()
        return False


def angle_errors(records, chi_model=0, chi_alpha=1.0):
    """Empirical-CDF errors of (chi, eps) records against the analytic CDFs of
    the polar-angle model (isotropic by default) and of the uniform azimuth:
    (eps_2 chi, eps_inf chi, eps_2 eps, eps_inf eps)."""
    rec = np.ascontiguousarray(records, dtype=np.float64).reshape(-1)
    out = np.zeros(4)
    lib().orc_angle_errors(_dp(rec), len(rec) // 2, int(chi_model), float(chi_alpha), _dp(out))
    return out


def cos_chi(chi_model, chi_alpha, xi):
    """cos F_pchi^{-1}(xi) of the polar-angle model (eq. chi_iso, eq. fpiv_ms, eq. vss)."""
    return lib().orc_cos_chi(int(chi_model), float(chi_alpha), float(xi))


def chi_cdf(chi_model, chi_alpha, chi):
    """F_pchi(chi) of the polar-angle model."""
    return lib().orc_chi_cdf(int(chi_model), float(chi_alpha), float(chi))
