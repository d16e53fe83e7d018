"""Thin Python binding of the HIP library (include/pic.h): argument marshalling only.

Every stage of the time step runs in the HIP kernels of ``libpic.so``; torch is
used only to allocate the device workspace and to name the stream.  Importing
this module loads the library and raises if it is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_EHIP, PIC_ENOCONV, PIC_ENONFINITE, PIC_ESTATE, PIC_ESPACE = 0, -1, -2, -3, -4, -5, -6
PIC_WARN_NAVG, PIC_WARN_GMAX = 1, 2
PIC_FP64, PIC_MIXED = 0, 1
PRECISION = {"fp64": PIC_FP64, "mixed": PIC_MIXED}
FAMILY = {"paper": 0, "cfg": 1}
SIGMA = {"poly": 0, "vhs": 1}
STATE_X, STATE_V, STATE_ID, STATE_CELL_START, STATE_RHO, STATE_PHI, STATE_E = range(7)


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pic error {code}: {msg}")
        self.code = code


class pic_problem(C.Structure):
    _fields_ = [
        ("family", C.c_int), ("L", C.c_double * 3), ("nphys", C.c_double), ("q", C.c_double),
        ("m", C.c_double), ("eps0", C.c_double), ("T", C.c_double), ("vbar", C.c_double),
        ("phibar", C.c_double), ("rho_amp", C.c_double), ("sigma_model", C.c_int),
        ("n_sigma", C.c_int), ("sigma_n", C.c_double * 3), ("sigma_ref", C.c_double),
        ("g_ref", C.c_double), ("omega", C.c_double), ("g_max", C.c_double),
        ("chi_model", C.c_int), ("field_to_particles", C.c_int), ("particles_to_field", C.c_int),
        ("collisions", C.c_int), ("isolate", C.c_int), ("chi_alpha", C.c_double),
        ("coding_error", C.c_int),
    ]


class pic_discretization(C.Structure):
    _fields_ = [("ncell", C.c_int * 3), ("n_particles", C.c_int64), ("dt", C.c_double),
                ("n_avg", C.c_int), ("cg_tol", C.c_double), ("cg_max_iter", C.c_int),
                ("poisson_op", C.c_int)]


class pic_error_norms(C.Structure):
    _fields_ = [("t", C.c_double), ("l2", C.c_double * 7), ("linf", C.c_double * 7)]


class pic_stats_t(C.Structure):
    _fields_ = [("step", C.c_int64), ("cg_iters", C.c_int), ("cg_relres", C.c_double),
                ("n_accepted", C.c_int64), ("n_gmax", C.c_int64),
                ("cg_blocks", C.c_int), ("cg_brick", C.c_int * 3),
                ("cg_members_per_launch", C.c_int)]


def _load():
    # torch's HIP runtime is loaded before this library's dependencies, so
    # that the process has one runtime whatever the caller imported first
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run python -m paper_2602_15130_amd.build)")
    L = C.CDLL(LIB_PATH)
    P, vp, i64 = C.POINTER, C.c_void_p, C.c_int64
    L.pic_workspace_size.argtypes = [P(pic_problem), P(pic_discretization), C.c_int, P(i64)]
    L.pic_init_manufactured.argtypes = [P(vp), P(pic_problem), P(pic_discretization), C.c_uint64,
                                        C.c_uint32, C.c_int, vp, i64, vp]
    L.pic_step.argtypes = [vp, C.c_int]
    L.pic_collide.argtypes = [vp, C.c_int, C.c_double, vp, vp, vp, i64, P(i64)]
    L.pic_errors.argtypes = [vp, P(pic_error_norms)]
    L.pic_stats.argtypes = [vp, P(pic_stats_t)]
    L.pic_get_state.argtypes = [vp, C.c_int, vp, i64]
    L.pic_set_state.argtypes = [vp, C.c_int, vp, i64]
    L.pic_ensemble_workspace_size.argtypes = [P(pic_problem), P(pic_discretization), C.c_int,
                                              C.c_int, P(i64)]
    L.pic_ensemble_init.argtypes = [P(vp), P(pic_problem), P(pic_discretization), C.c_uint64,
                                    C.c_uint32, C.c_int, C.c_int, vp, i64, vp]
    L.pic_ensemble_errors.argtypes = [vp, P(pic_error_norms)]
    L.pic_ensemble_get_state.argtypes = [vp, C.c_int, C.c_int, vp, i64]
    L.pic_errors_noalloc.argtypes = [vp, P(pic_error_norms)]
    L.pic_timing_enable.argtypes = [vp, C.c_int]
    L.pic_timing_stages.argtypes = [vp, C.c_uint32]
    L.pic_timing_read.argtypes = [vp, P(C.c_double), P(i64)]
    L.pic_angle_buffer_bytes.argtypes = [i64]
    L.pic_angle_buffer_bytes.restype = i64
    L.pic_angle_log.argtypes = [vp, vp, i64]
    L.pic_angle_errors.argtypes = [vp, P(C.c_double), P(i64)]
    L.pic_checkpoint_bytes.argtypes = [vp, P(i64)]
    L.pic_checkpoint_save.argtypes = [vp, vp, i64]
    L.pic_checkpoint_load.argtypes = [vp, vp, i64]
    L.pic_destroy.argtypes = [vp]
    L.pic_destroy.restype = None
    L.pic_last_error.argtypes = [vp]
    L.pic_last_error.restype = C.c_char_p
    return L


lib = _load()

EXPORTED = ("pic_workspace_size", "pic_init_manufactured", "pic_step", "pic_collide", "pic_errors",
            "pic_errors_noalloc", "pic_stats", "pic_get_state", "pic_set_state", "pic_timing_enable", "pic_timing_stages", "pic_timing_read",
            "pic_destroy",
            "pic_angle_buffer_bytes", "pic_angle_log", "pic_angle_errors",
            "pic_checkpoint_bytes", "pic_checkpoint_save", "pic_checkpoint_load",
            "pic_ensemble_workspace_size", "pic_ensemble_init", "pic_ensemble_errors",
            "pic_ensemble_get_state", "pic_use_graphs", "pic_last_error")
STAGES = ("collide", "kick", "drift", "sort", "deposit", "cg", "gradient", "particle")


def make_problem(p: dict) -> pic_problem:
    s = pic_problem()
    s.family = FAMILY[p["family"]]
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
    s.coding_error = int(p.get("coding_error", 0))
    for k in ("field_to_particles", "particles_to_field", "collisions", "isolate"):
        setattr(s, k, int(p[k]))
    return s


def make_disc(d: dict) -> pic_discretization:
    s = pic_discretization()
    s.ncell = (C.c_int * 3)(*d["nc"])
    s.n_particles = int(d["np"])
    s.dt = float(d["dt"])
    s.n_avg = int(d["navg"])
    s.cg_tol = float(d["cg_tol"])
    s.cg_max_iter = int(d["cg_max_iter"])
    s.poisson_op = int(d.get("poisson_op", 0))
    return s


def _err(ctx):
    m = lib.pic_last_error(ctx)
    return m.decode() if m else ""


def _check(code, ctx=None):
    if code < 0:
        raise PicError(code, _err(ctx))
    return code


# ---- the C ABI, one Python function per entry point -------------------------
def pic_workspace_size(prob: dict, disc: dict, precision: str = "fp64") -> int:
    b = C.c_int64()
    _check(lib.pic_workspace_size(C.byref(make_problem(prob)), C.byref(make_disc(disc)),
                                  PRECISION[precision], C.byref(b)))
    return b.value


def pic_init_manufactured(prob, disc, seed, replicate, precision, workspace_ptr, workspace_bytes,
                          stream_ptr):
    ctx = C.c_void_p()
    st = lib.pic_init_manufactured(C.byref(ctx), C.byref(make_problem(prob)),
                                   C.byref(make_disc(disc)), int(seed), int(replicate),
                                   PRECISION[precision], C.c_void_p(workspace_ptr),
                                   int(workspace_bytes), C.c_void_p(stream_ptr))
    _check(st, None)
    return ctx, st


def pic_step(ctx, n_steps: int):
    return _check(lib.pic_step(ctx, int(n_steps)), ctx)


def pic_collide(ctx, call, t, dv_avg_ptr, dv_src_ptr, pairlog_ptr=0, pairlog_cap=0):
    """Number of candidate pairs and the status (PIC_OK or a PIC_WARN_* code)."""
    n = C.c_int64()
    st = _check(lib.pic_collide(ctx, int(call), float(t), C.c_void_p(dv_avg_ptr),
                                C.c_void_p(dv_src_ptr), C.c_void_p(pairlog_ptr or None),
                                int(pairlog_cap), C.byref(n)), ctx)
    return n.value, st


def pic_errors(ctx) -> dict:
    e = pic_error_norms()
    st = _check(lib.pic_errors(ctx, C.byref(e)), ctx)
    return {"t": e.t, "l2": np.array(list(e.l2)), "linf": np.array(list(e.linf)), "status": st}


def pic_stats(ctx) -> dict:
    s = pic_stats_t()
    _check(lib.pic_stats(ctx, C.byref(s)), ctx)
    return {"step": s.step, "cg_iters": s.cg_iters, "cg_relres": s.cg_relres,
            "n_accepted": s.n_accepted, "n_gmax": s.n_gmax,
            "cg_blocks": s.cg_blocks, "cg_brick": list(s.cg_brick),
            "cg_members_per_launch": s.cg_members_per_launch}


def pic_errors_noalloc(ctx) -> dict:
    """pic_errors with its partial sums in the library's static scratch."""
    e = pic_error_norms()
    st = _check(lib.pic_errors_noalloc(ctx, C.byref(e)), ctx)
    return {"t": e.t, "l2": np.array(list(e.l2)), "linf": np.array(list(e.linf)), "status": st}


def pic_ensemble_workspace_size(prob: dict, disc: dict, precision: str, members: int) -> int:
    b = C.c_int64()
    _check(lib.pic_ensemble_workspace_size(C.byref(make_problem(prob)), C.byref(make_disc(disc)),
                                           PRECISION[precision], int(members), C.byref(b)))
    return b.value


def pic_ensemble_init(prob, disc, seed, first_replicate, members, precision, workspace_ptr,
                      workspace_bytes, stream_ptr):
    ctx = C.c_void_p()
    st = lib.pic_ensemble_init(C.byref(ctx), C.byref(make_problem(prob)), C.byref(make_disc(disc)),
                               int(seed), int(first_replicate), int(members),
                               PRECISION[precision], C.c_void_p(workspace_ptr),
                               int(workspace_bytes), C.c_void_p(stream_ptr))
    _check(st, None)
    return ctx, st


def pic_ensemble_errors(ctx, members: int) -> dict:
    e = (pic_error_norms * members)()
    st = _check(lib.pic_ensemble_errors(ctx, e), ctx)
    return {"t": e[0].t, "l2": np.array([list(x.l2) for x in e]),
            "linf": np.array([list(x.linf) for x in e]), "status": st}


def pic_ensemble_get_state(ctx, member: int, item: int, out: np.ndarray):
    _check(lib.pic_ensemble_get_state(ctx, int(member), int(item), out.ctypes.data, out.nbytes), ctx)
    return out


def pic_get_state(ctx, item: int, out: np.ndarray):
    _check(lib.pic_get_state(ctx, int(item), out.ctypes.data, out.nbytes), ctx)
    return out


def pic_set_state(ctx, item: int, src: np.ndarray):
    src = np.ascontiguousarray(src, dtype=np.float64)
    return _check(lib.pic_set_state(ctx, int(item), src.ctypes.data, src.nbytes), ctx)


def pic_use_graphs(ctx, enable: bool):
    return _check(lib.pic_use_graphs(ctx, int(bool(enable))), ctx)


def pic_timing_enable(ctx, enable: bool):
    return _check(lib.pic_timing_enable(ctx, int(bool(enable))), ctx)


def pic_timing_stages(ctx, stages):
    """Time only the named stages (an empty list stops timing)."""
    mask = 0
    for name in stages:
        mask |= 1 << STAGES.index(name)
    return _check(lib.pic_timing_stages(ctx, mask), ctx)


def pic_timing_read(ctx) -> dict:
    ms = (C.c_double * len(STAGES))()
    n = (C.c_int64 * len(STAGES))()
    _check(lib.pic_timing_read(ctx, ms, n), ctx)
    return {name: (ms[i], n[i]) for i, name in enumerate(STAGES)}


def pic_angle_buffer_bytes(capacity: int) -> int:
    return lib.pic_angle_buffer_bytes(int(capacity))


def pic_angle_log(ctx, buffer_ptr, capacity: int):
    _check(lib.pic_angle_log(ctx, buffer_ptr, int(capacity)), ctx)


def pic_angle_errors(ctx):
    out = (C.c_double * 4)()
    n = C.c_int64()
    _check(lib.pic_angle_errors(ctx, out, C.byref(n)), ctx)
    return list(out), n.value


def pic_checkpoint_save(ctx) -> bytes:
    n = C.c_int64()
    _check(lib.pic_checkpoint_bytes(ctx, C.byref(n)), ctx)
    buf = C.create_string_buffer(n.value)
    _check(lib.pic_checkpoint_save(ctx, buf, n.value), ctx)
    return buf.raw


def pic_checkpoint_load(ctx, data: bytes):
    buf = C.create_string_buffer(data, len(data))
    _check(lib.pic_checkpoint_load(ctx, buf, len(data)), ctx)


def pic_destroy(ctx):
    lib.pic_destroy(ctx)


# ---- convenience wrapper -----------------------------------------------------
class Sim:
    """One simulation on a GPU: torch allocates the workspace, the library does the rest."""

    def __init__(self, prob: dict, disc: dict, seed: int = 1, replicate: int = 0,
                 precision: str = "fp64", device: str = "cuda:0", stream=None):
        import torch

        self.prob, self.disc, self.precision = prob, disc, precision
        self.np = int(disc["np"])
        self.nn = int(np.prod(disc["nc"]))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = pic_workspace_size(prob, disc, precision)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        ptr = (base + 255) // 256 * 256
        # held by the instance so that teardown at interpreter exit still finds it
        self._destroy = lib.pic_destroy
        self.ctx, self.init_status = pic_init_manufactured(
            prob, disc, seed, replicate, precision, ptr, nbytes, self.stream.cuda_stream)

    def close(self):
        """Release the context (pic_destroy synchronises its stream); the
        workspace is freed with this object."""
        ctx = getattr(self, "ctx", None)
        destroy = getattr(self, "_destroy", None)
        if ctx and destroy is not None:
            destroy(ctx)
        self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP calls while the interpreter (and with it the runtime) shuts
        # down: contexts still open then are left to the process exit (the
        # check is bound at definition, module globals may be gone by then)
        if _finalizing():
            return
        self.close()

    def step(self, n: int = 1):
        pic_step(self.ctx, n)

    def collide(self, call: int, t: float, pairlog_cap: int = 0):
        import torch

        dv = torch.zeros(3 * self.np, dtype=torch.float64, device=self.device)
        src = torch.zeros(3 * self.np, dtype=torch.float64, device=self.device)
        log = torch.zeros(max(1, pairlog_cap) * 7, dtype=torch.int64, device=self.device)
        n, self.collide_status = pic_collide(self.ctx, call, t, dv.data_ptr(), src.data_ptr(),
                                             log.data_ptr() if pairlog_cap else 0, pairlog_cap)
        pairs = log[: 7 * min(n, pairlog_cap)].view(-1, 7).cpu().numpy() if pairlog_cap else None
        return (dv.view(3, -1).cpu().numpy(), src.view(3, -1).cpu().numpy(), pairs, n)

    def errors(self) -> dict:
        return pic_errors(self.ctx)

    def checkpoint(self) -> bytes:
        return pic_checkpoint_save(self.ctx)

    def restore(self, data: bytes):
        pic_checkpoint_load(self.ctx, data)

    def angle_log(self, capacity: int):
        """Record (chi, eps) of every accepted collision from now on, up to `capacity`."""
        import torch

        nbytes = pic_angle_buffer_bytes(capacity)
        self._ang = torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ang.data_ptr() + 255) // 256 * 256 if capacity > 0 else 0
        self._ang_ptr, self._ang_cap = ptr, capacity
        pic_angle_log(self.ctx, ptr, capacity)

    def angle_errors(self):
        """(eps_2 chi, eps_inf chi, eps_2 eps, eps_inf eps), number of records."""
        return pic_angle_errors(self.ctx)

    def angle_records(self, n: int) -> np.ndarray:
        """The first n records as an [n, 2] host array (chi, eps)."""
        import torch

        self.stream.synchronize()
        off = self._ang_ptr - self._ang.data_ptr()
        raw = self._ang[off: off + 16 * n].view(torch.float64)
        return raw.cpu().numpy().reshape(n, 2)

    def use_graphs(self, enable: bool = True):
        """Replay recorded two-step graphs in pic_step (bitwise the same results)."""
        pic_use_graphs(self.ctx, enable)

    def timing(self, enable: bool):
        pic_timing_enable(self.ctx, enable)

    def timing_stages(self, stages):
        pic_timing_stages(self.ctx, stages)

    def timing_read(self) -> dict:
        return pic_timing_read(self.ctx)

    def stats(self) -> dict:
        return pic_stats(self.ctx)

    def set(self, item: int, values: np.ndarray):
        """Replace positions (re-sort and field solve follow) or velocities."""
        return pic_set_state(self.ctx, item, values)

    def get(self, item: int) -> np.ndarray:
        if item in (STATE_X, STATE_V):
            out = np.zeros((3, self.np))
        elif item == STATE_ID:
            out = np.zeros(self.np, dtype=np.int64)
        elif item == STATE_CELL_START:
            out = np.zeros(self.nn + 1, dtype=np.int64)
        elif item == STATE_E:
            out = np.zeros((3, self.nn))
        else:
            out = np.zeros(self.nn)
        return pic_get_state(self.ctx, item, out)


class Ensemble:
    """`members` replicates of one problem run together (one launch per stage
    for all of them); torch allocates the workspace, the library does the rest."""

    def __init__(self, prob: dict, disc: dict, seed: int = 1, first_replicate: int = 0,
                 members: int = 1, precision: str = "mixed", device: str = "cuda:0", stream=None):
        import torch

        self.prob, self.disc, self.precision, self.members = prob, disc, precision, int(members)
        self.np = int(disc["np"])
        self.nn = int(np.prod(disc["nc"]))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = pic_ensemble_workspace_size(prob, disc, precision, members)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ws.data_ptr() + 255) // 256 * 256
        self._destroy = lib.pic_destroy
        self.ctx, self.init_status = pic_ensemble_init(prob, disc, seed, first_replicate, members,
                                                       precision, ptr, nbytes,
                                                       self.stream.cuda_stream)

    close = Sim.close
    __enter__ = Sim.__enter__
    __exit__ = Sim.__exit__
    __del__ = Sim.__del__
    step = Sim.step
    stats = Sim.stats
    use_graphs = Sim.use_graphs
    timing = Sim.timing
    timing_stages = Sim.timing_stages
    timing_read = Sim.timing_read

    def errors(self) -> dict:
        """Norms of every member: l2 and linf as [members, 7] arrays."""
        return pic_ensemble_errors(self.ctx, self.members)

    def get(self, member: int, item: int) -> np.ndarray:
        if item in (STATE_X, STATE_V):
            out = np.zeros((3, self.np))
        elif item == STATE_ID:
            out = np.zeros(self.np, dtype=np.int64)
        elif item == STATE_CELL_START:
            out = np.zeros(self.nn + 1, dtype=np.int64)
        elif item == STATE_E:
            out = np.zeros((3, self.nn))
        else:
            out = np.zeros(self.nn)
        return pic_ensemble_get_state(self.ctx, member, item, out)
