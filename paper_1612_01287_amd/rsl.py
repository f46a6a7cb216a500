"""ctypes binding of librsl (include/rsl.h) with torch tensors as device memory.

Argument marshalling only: every step of the R-SLB path runs in the HIP
kernels of librsl.so.  The library must have been built (``build.py``); a
missing library raises at import, there is no fallback.
"""
import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsl.so")
HEADER = os.path.join(HERE, "..", "include", "rsl.h")

if not os.path.exists(LIB_PATH):
    raise ImportError("librsl.so is not built: run `python -m paper_1612_01287_amd.build` "
                      "(or __graft_entry__.build()) first")

_lib = ctypes.CDLL(LIB_PATH)


def _constants():
    """#define RSL_* integer constants parsed from the public header."""
    out = {}
    with open(HEADER) as fh:
        for line in fh:
            m = re.match(r"#define\s+(RSL_\w+)\s+\(?(-?\d+)\)?", line)
            if m:
                out[m.group(1)] = int(m.group(2))
    return out


C = _constants()
globals().update(C)

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


class Problem(ctypes.Structure):
    """Mirror of struct rsl_problem."""
    _fields_ = [("problem", ctypes.c_int), ("nz", ctypes.c_int), ("dtype", ctypes.c_int),
                ("bc", ctypes.c_int), ("tau_mode", ctypes.c_int), ("gas", ctypes.c_int),
                ("flags", ctypes.c_int), ("reserved", ctypes.c_int),
                ("z_lo", ctypes.c_double), ("z_hi", ctypes.c_double),
                ("n_L", ctypes.c_double), ("T_L", ctypes.c_double),
                ("n_R", ctypes.c_double), ("T_R", ctypes.c_double),
                ("tau_r", ctypes.c_double), ("tau_aw0", ctypes.c_double),
                ("lambda_ref", ctypes.c_double), ("kappa", ctypes.c_double)]


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


_sig("rsl_make_quadrature", ctypes.c_int,
     [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
      ctypes.POINTER(_vp)])
_sig("rsl_free_quadrature", None, [_vp])
_sig("rsl_quad_table", ctypes.c_int, [_vp, ctypes.c_int, _dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)])
_sig("rsl_pitch", ctypes.c_int, [ctypes.c_int])
_sig("rsl_max_dt", ctypes.c_int, [_vp, ctypes.POINTER(Problem), _dp, _dp])
_sig("rsl_sizes", ctypes.c_int, [_vp, ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_size_t)])
_sig("rsl_init", ctypes.c_int, [_vp, ctypes.POINTER(Problem), _vp, _vp, _vp])
_sig("rsl_step", ctypes.c_int, [_vp, ctypes.POINTER(Problem), _vp, _vp, _dp, ctypes.c_double,
                                ctypes.c_int, _vp])
_sig("rsl_moments", ctypes.c_int, [_vp, ctypes.POINTER(Problem), _vp, _vp, _vp, ctypes.c_int, _vp])
_sig("rsl_step_imex", ctypes.c_int, [_vp, ctypes.POINTER(Problem), _vp, _vp, _dp, ctypes.c_double,
                                     ctypes.c_int, _vp])
_sig("rsl_status", ctypes.c_int, [_vp, ctypes.POINTER(Problem), _vp, _vp])
_sig("rsl_last_error", ctypes.c_char_p, [])

MOMENT_FIELDS = ("N0", "Nz", "T00", "T0z", "Tzz", "n", "E", "P", "T", "beta", "lambda", "q", "Pi")


class RslError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("rsl error %d: %s" % (code, msg))
        self.code = code


def check(rc):
    if rc != 0:
        raise RslError(rc, _lib.rsl_last_error().decode())
    return rc


def lib():
    return _lib


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Quadrature:
    """R-SLB(N_Omega; Q_xi) velocity set with Q_L radial nodes (owned library handle)."""

    def __init__(self, QL, Q, NOm, T0=1.0, host_only=False):
        h = _vp()
        check(_lib.rsl_make_quadrature(QL, Q, 1, NOm, float(T0),
                                       C["RSL_QUAD_HOST_ONLY"] if host_only else 0, ctypes.byref(h)))
        self._h = h
        self.QL, self.Q, self.NOm, self.T0 = QL, Q, NOm, float(T0)
        self.V = QL * Q

    @property
    def handle(self):
        return self._h

    def table(self, which):
        import numpy as np
        cnt = ctypes.c_int(0)
        check(_lib.rsl_quad_table(self._h, which, None, 0, ctypes.byref(cnt)))
        out = np.zeros(cnt.value)
        check(_lib.rsl_quad_table(self._h, which, out.ctypes.data_as(_dp), cnt.value, None))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.rsl_free_quadrature(h)
            self._h = None


def max_dt(quad, problem):
    """(CFL bound, stiffness bound) on dt that rsl_step's guards apply (host only)."""
    a, b = ctypes.c_double(0), ctypes.c_double(0)
    check(_lib.rsl_max_dt(quad.handle, ctypes.byref(problem), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def make_problem(kind="sod", nz=400, dtype="f64", bc="outflow", tau_mode="const", gas="ideal",
                 z_lo=-0.5, z_hi=0.5, nL=1.0, TL=1.0, nR=0.4, TR=0.8, tau_r=1e-3, tau_aw0=0.0,
                 lambda_ref=1.0, kappa=0.0, force=False, imex=False):
    p = Problem()
    p.problem = C["RSL_SOD"] if kind == "sod" else C["RSL_BJORKEN"]
    p.nz = nz if kind == "sod" else 1
    p.dtype = C["RSL_F64"] if dtype == "f64" else C["RSL_F32"]
    p.bc = C["RSL_BC_OUTFLOW"] if bc == "outflow" else C["RSL_BC_EQ"]
    p.tau_mode = {"const": C["RSL_TAU_CONST"], "etas": C["RSL_TAU_ETAS"], "inf": C["RSL_TAU_INF"]}[tau_mode]
    p.gas = C["RSL_GAS_IDEAL"] if gas == "ideal" else C["RSL_GAS_PARTON"]
    p.flags = (C["RSL_FLAG_FORCE_UNSTABLE"] if force else 0) | (C["RSL_FLAG_IMEX"] if imex else 0)
    p.z_lo, p.z_hi = z_lo, z_hi
    p.n_L, p.T_L, p.n_R, p.T_R = nL, TL, nR, TR
    p.tau_r, p.tau_aw0, p.lambda_ref, p.kappa = tau_r, tau_aw0, lambda_ref, kappa
    return p


class Instance:
    """One problem instance: caller-side buffers (torch uint8 tensors on the GPU)
    for the state f and the work area, plus the host-side time."""

    def __init__(self, quad, problem, device="cuda"):
        self.quad, self.p = quad, problem
        fb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        check(_lib.rsl_sizes(quad.handle, ctypes.byref(problem), ctypes.byref(fb), ctypes.byref(wb)))
        self.f_buf = torch.empty(fb.value, dtype=torch.uint8, device=device)
        self.work = torch.empty(wb.value, dtype=torch.uint8, device=device)
        self.t = 0.0
        self.nz = problem.nz
        self.pitch = _lib.rsl_pitch(problem.nz) if problem.problem == C["RSL_SOD"] else 1
        self.tdtype = torch.float64 if problem.dtype == C["RSL_F64"] else torch.float32

    def _ptrs(self):
        return ctypes.c_void_p(self.f_buf.data_ptr()), ctypes.c_void_p(self.work.data_ptr())

    def init(self, t0=0.0, stream=None):
        f, w = self._ptrs()
        check(_lib.rsl_init(self.quad.handle, ctypes.byref(self.p), f, w, _stream(stream)))
        self.t = float(t0)

    def step(self, dt, nsteps=1, stream=None):
        f, w = self._ptrs()
        t = ctypes.c_double(self.t)
        check(_lib.rsl_step(self.quad.handle, ctypes.byref(self.p), f, w, ctypes.byref(t), float(dt),
                            int(nsteps), _stream(stream)))
        self.t = t.value

    def step_imex(self, dt, nsteps=1, stream=None):
        """rsl_step_imex: implicit-explicit steps (binary64 Sod instances)."""
        f, w = self._ptrs()
        t = ctypes.c_double(self.t)
        check(_lib.rsl_step_imex(self.quad.handle, ctypes.byref(self.p), f, w, ctypes.byref(t), float(dt),
                                 int(nsteps), _stream(stream)))
        self.t = t.value

    def f(self):
        """[V, nz] view of the state (no copy)."""
        es = 8 if self.tdtype == torch.float64 else 4
        n = self.f_buf.numel() // es
        flat = self.f_buf.view(self.tdtype)[:n]
        return flat[: self.quad.V * self.pitch].view(self.quad.V, self.pitch)[:, : self.nz]

    def set_f(self, values):
        self.f().copy_(torch.as_tensor(values, dtype=self.tdtype))

    def moments(self, stream=None, fields=None):
        """[nz, fields] per-cell fields (RSL_MOM_ALL by default, or RSL_MOM_RAW5)."""
        fields = C["RSL_MOM_ALL"] if fields is None else int(fields)
        out = torch.empty((self.nz, fields), dtype=torch.float64, device=self.f_buf.device)
        f, w = self._ptrs()
        check(_lib.rsl_moments(self.quad.handle, ctypes.byref(self.p), f, w, ctypes.c_void_p(out.data_ptr()),
                               fields, _stream(stream)))
        return out

    def status(self, stream=None):
        _, w = self._ptrs()
        return _lib.rsl_status(self.quad.handle, ctypes.byref(self.p), w, _stream(stream))


_sig("rsl_batch_create", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(Problem), _dp, ctypes.c_int,
                                        ctypes.POINTER(_vp)])
_sig("rsl_batch_free", None, [_vp])
_sig("rsl_batch_sizes", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)])
_sig("rsl_batch_offset", ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)])
_sig("rsl_batch_time", ctypes.c_int, [_vp, ctypes.c_int, _dp])
_sig("rsl_batch_init", ctypes.c_int, [_vp, _vp, _vp, _vp])
_sig("rsl_batch_step", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp])
_sig("rsl_batch_step_imex", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp])
_sig("rsl_batch_stage", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp])
_sig("rsl_batch_graph_step", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp])
_sig("rsl_batch_set_path", ctypes.c_int, [_vp, ctypes.c_int])
_sig("rsl_batch_groups", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.c_int])
_sig("rsl_batch_moments", ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, _vp])
_sig("rsl_batch_status", ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int)])
_sig("rsl_batch_instance_status", ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int)])
_ip = ctypes.POINTER(ctypes.c_int)
_sig("rsl_stage_variant", ctypes.c_int, [ctypes.c_int, _ip, _ip, _ip, _ip, _ip, _ip])
_sig("rsl_batch_variant", ctypes.c_int, [_vp, ctypes.c_int, _ip, _ip])
_sig("rsl_batch_set_variant", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int])
_sig("rsl_batch_autotune", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, _ip])

N_CLASSES = 7


def stage_variants():
    """[(waves, velocities per lane, lanes per velocity, largest V, cell-kernel
    waves (0: fused form), form (0 fused, 1 two-kernel, 2 loop))] of every
    stage-kernel variant, by id."""
    out = []
    while True:
        r = [ctypes.c_int() for _ in range(6)]
        if _lib.rsl_stage_variant(len(out), *[ctypes.byref(x) for x in r]) != 0:
            return out
        out.append(tuple(x.value for x in r))


class Batch:
    """Many instances (one kind, one dtype) advanced together; see rsl_batch_* in rsl.h."""

    def __init__(self, quads, problems, dts, device="cuda"):
        n = len(problems)
        self.quads = list(quads)            # keep the handles alive
        self.problems = (Problem * n)(*problems)
        qarr = (_vp * n)(*[q.handle for q in self.quads])
        dtarr = (ctypes.c_double * n)(*[float(x) for x in dts])
        h = _vp()
        check(_lib.rsl_batch_create(qarr, self.problems, dtarr, n, ctypes.byref(h)))
        self._h = h
        self.n = n
        fb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        check(_lib.rsl_batch_sizes(h, ctypes.byref(fb), ctypes.byref(wb)))
        self.f_buf = torch.empty(fb.value, dtype=torch.uint8, device=device)
        self.work = torch.empty(wb.value, dtype=torch.uint8, device=device)
        self.tdtype = torch.float64 if problems[0].dtype == C["RSL_F64"] else torch.float32

    def _ptrs(self):
        return ctypes.c_void_p(self.f_buf.data_ptr()), ctypes.c_void_p(self.work.data_ptr())

    def init(self, stream=None):
        f, w = self._ptrs()
        check(_lib.rsl_batch_init(self._h, f, w, _stream(stream)))

    def step(self, nsteps=1, stream=None):
        f, w = self._ptrs()
        check(_lib.rsl_batch_step(self._h, f, w, int(nsteps), _stream(stream)))

    def step_imex(self, nsteps=1, stream=None):
        """rsl_batch_step_imex: implicit-explicit steps of every Sod instance."""
        f, w = self._ptrs()
        check(_lib.rsl_batch_step_imex(self._h, f, w, int(nsteps), _stream(stream)))

    def graph_step(self, nsteps=1, stream=None):
        """nsteps steps replayed from a captured HIP graph (needs a non-default stream)."""
        f, w = self._ptrs()
        check(_lib.rsl_batch_graph_step(self._h, f, w, int(nsteps), _stream(stream)))

    def set_path(self, path):
        """Bjorken batches: -1 automatic, 0 vector units, 1 matrix cores."""
        check(_lib.rsl_batch_set_path(self._h, int(path)))

    def groups(self):
        """Instances per matrix-core group of a Bjorken batch, in launch order."""
        n = ctypes.c_int(0)
        check(_lib.rsl_batch_groups(self._h, ctypes.byref(n), None, 0))
        out = (ctypes.c_int * max(n.value, 1))()
        check(_lib.rsl_batch_groups(self._h, ctypes.byref(n), out, n.value))
        return list(out)[:n.value]

    def variant(self, cls):
        """(variant id or -1 for an empty class, largest V of the class)."""
        v, mv = ctypes.c_int(), ctypes.c_int()
        check(_lib.rsl_batch_variant(self._h, int(cls), ctypes.byref(v), ctypes.byref(mv)))
        return v.value, mv.value

    def set_variant(self, cls, var):
        check(_lib.rsl_batch_set_variant(self._h, int(cls), int(var)))

    def autotune(self, reps=5, stream=None):
        """Times every fitting kernel variant per class and keeps the fastest;
        returns the chosen ids per class (-1: empty class)."""
        f, w = self._ptrs()
        out = (ctypes.c_int * N_CLASSES)()
        check(_lib.rsl_batch_autotune(self._h, f, w, int(reps), _stream(stream), out))
        return list(out)

    def stage(self, s, stream=None):
        f, w = self._ptrs()
        check(_lib.rsl_batch_stage(self._h, f, w, int(s), _stream(stream)))

    def time(self, i):
        t = ctypes.c_double(0)
        check(_lib.rsl_batch_time(self._h, i, ctypes.byref(t)))
        return t.value

    def f(self, i):
        """[V, nz] view of instance i's state (no copy)."""
        off = ctypes.c_size_t(0)
        check(_lib.rsl_batch_offset(self._h, i, ctypes.byref(off)))
        p, q = self.problems[i], self.quads[i]
        es = 8 if self.tdtype == torch.float64 else 4
        nz = p.nz
        pitch = _lib.rsl_pitch(nz) if p.problem == C["RSL_SOD"] else 1
        flat = self.f_buf[off.value: off.value + q.V * pitch * es].view(self.tdtype)
        return flat.view(q.V, pitch)[:, :nz]

    def moments(self, stream=None, fields=None):
        fields = C["RSL_MOM_ALL"] if fields is None else int(fields)
        rows = sum(p.nz if p.problem == C["RSL_SOD"] else 1 for p in self.problems)
        out = torch.empty((rows, fields), dtype=torch.float64, device=self.f_buf.device)
        f, w = self._ptrs()
        check(_lib.rsl_batch_moments(self._h, f, w, ctypes.c_void_p(out.data_ptr()), fields, _stream(stream)))
        return out

    def status(self, stream=None):
        _, w = self._ptrs()
        bad = ctypes.c_int(-1)
        rc = _lib.rsl_batch_status(self._h, w, _stream(stream), ctypes.byref(bad))
        return rc, bad.value

    def instance_status(self, stream=None):
        """Status code (0 or RSL_ENONFINITE) of every instance."""
        _, w = self._ptrs()
        out = (ctypes.c_int * self.n)()
        check(_lib.rsl_batch_instance_status(self._h, w, _stream(stream), out))
        return list(out)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.rsl_batch_free(h)
            self._h = None


_sig("rsl_window_integral", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_int, _vp, _vp])
_sig("rsl_sod_eps", ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp])
_sig("rsl_bjorken_l2", ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_double, _vp, _vp])


def window_integral(m, dz, row_lo, row_hi, stream=None):
    """[ncols] dz * sum of rows row_lo..row_hi-1 of the [nrows, ncols] fp64 table m (device)."""
    out = torch.empty(m.shape[1], dtype=torch.float64, device=m.device)
    check(_lib.rsl_window_integral(_p(m), m.shape[0], m.shape[1], float(dz), int(row_lo), int(row_hi), _p(out),
                                   _stream(stream)))
    return out


def sod_eps(m, ref, stream=None):
    """[eps_n, eps_T, eps_gamma, eps] of two [nz, RSL_MOM_ALL] moment tables (eq. eps_def)."""
    out = torch.empty(4, dtype=torch.float64, device=m.device)
    check(_lib.rsl_sod_eps(_p(m), _p(ref), m.shape[0], _p(out), _stream(stream)))
    return out


def bjorken_l2(hist, ref, dtau, stream=None):
    """[L2(n), L2(T), L2(P), L2(Pi), max] of two [nsamples, RSL_MOM_ALL] histories (eq. bjork_L2)."""
    out = torch.empty(5, dtype=torch.float64, device=hist.device)
    check(_lib.rsl_bjorken_l2(_p(hist), _p(ref), hist.shape[0], float(dtau), _p(out), _stream(stream)))
    return out


_u16p = ctypes.c_void_p
_sig("rsl_mlp_features", ctypes.c_int, [_vp, ctypes.POINTER(Problem), _vp, ctypes.c_double, _vp, _vp, _vp, _vp])
_sig("rsl_mlp_to_bf16", ctypes.c_int, [_vp, _vp, _vp])
_sig("rsl_mlp_forward", ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp])
_sig("rsl_mlp_backward", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp])
_sig("rsl_mlp_backward_work", ctypes.c_size_t, [ctypes.c_int])
_sig("rsl_mlp_adam", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, _vp])
_sig("rsl_mlp_tmunu", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp])
_sig("rsl_mlp_guard", ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp])

MLP_SHAPES = (("W1", (81, 128)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)), ("W3", (128, 3)), ("b3", (3,)))


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class MLP:
    """The learned correction network: fp32 master parameters, bf16 compute copy
    and Adam state on the GPU (layout of rsl.h)."""

    def __init__(self, params=None, device="cuda"):
        n = C["RSL_MLP_NPARAM"]
        self.params = torch.zeros(n, dtype=torch.float32, device=device)
        if params is not None:
            self.params.copy_(torch.as_tensor(params, dtype=torch.float32))
        self.pb = torch.zeros(n, dtype=torch.int16, device=device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self._work = None                   # backward partial gradients (rsl_mlp_backward_work floats)
        self.step_count = 0
        self.refresh()

    def refresh(self, stream=None):
        check(_lib.rsl_mlp_to_bf16(_p(self.params), _p(self.pb), _stream(stream)))

    def forward(self, x, keep=False, stream=None):
        n = x.shape[0]
        y = torch.empty((n, 3), dtype=torch.float32, device=x.device)
        h1 = h2 = None
        if keep:
            h1 = torch.empty((n, 128), dtype=torch.int16, device=x.device)
            h2 = torch.empty((n, 128), dtype=torch.int16, device=x.device)
        check(_lib.rsl_mlp_forward(_p(self.pb), _p(x), n, _p(y), _p(h1), _p(h2), _stream(stream)))
        return (y, h1, h2) if keep else y

    def backward(self, x, h1, h2, y, t, stream=None):
        need = _lib.rsl_mlp_backward_work(x.shape[0])
        if self._work is None or self._work.numel() < need:
            self._work = torch.empty(need, dtype=torch.float32, device=self.params.device)
        check(_lib.rsl_mlp_backward(_p(self.pb), _p(x), _p(h1), _p(h2), _p(y), _p(t), x.shape[0], _p(self.grad),
                                    _p(self._work), _stream(stream)))
        return self.grad

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        check(_lib.rsl_mlp_adam(_p(self.params), _p(self.grad), _p(self.m), _p(self.v), _p(self.pb),
                                self.step_count, lr, b1, b2, eps, _stream(stream)))

    def unpack(self):
        """dict of numpy arrays in the oracle's naming (fp32 master copy)."""
        import numpy as np
        flat = self.params.cpu().numpy().astype(np.float64)
        out, o = {}, 0
        for name, shp in MLP_SHAPES:
            k = int(np.prod(shp))
            out[name] = flat[o:o + k].reshape(shp)
            o += k
        return out

    @staticmethod
    def pack(P):
        import numpy as np
        return np.concatenate([np.asarray(P[name], dtype=np.float64).ravel() for name, _ in MLP_SHAPES])


def features(quad, problem, f_buf, log_tau, shift=None, scale=None, stream=None):
    """[nz, 81] fp32 features of one Sod instance's state buffer, standardised
    as (x - shift) / scale when shift and scale ([81] fp32 device tensors) are given."""
    out = torch.empty((problem.nz, 81), dtype=torch.float32, device=f_buf.device)
    check(_lib.rsl_mlp_features(quad.handle, ctypes.byref(problem), _p(f_buf), float(log_tau), _p(shift), _p(scale),
                                _p(out), _stream(stream)))
    return out


def tmunu_targets(m_lo, m_hi, stream=None):
    n = m_lo.shape[0]
    t = torch.empty((n, 3), dtype=torch.float32, device=m_lo.device)
    check(_lib.rsl_mlp_tmunu(_p(m_lo), _p(m_hi), None, n, 0, _p(t), None, _stream(stream)))
    return t


def tmunu_correct(m_lo, y, stream=None):
    n = m_lo.shape[0]
    out = torch.empty((n, 3), dtype=torch.float64, device=m_lo.device)
    check(_lib.rsl_mlp_tmunu(_p(m_lo), None, _p(y), n, 1, None, _p(out), _stream(stream)))
    return out


def guard(x, lo, hi, stream=None):
    flag = torch.zeros(1, dtype=torch.int32, device=x.device)
    check(_lib.rsl_mlp_guard(_p(x), x.shape[0], _p(lo), _p(hi), _p(flag), _stream(stream)))
    return int(flag.item()) != 0


# ------------------------------------------- velocity sets with azimuthal nodes

_sig("rsl_make_quadrature3", ctypes.c_int,
     [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(_vp)])
_sig("rsl_free_quadrature3", None, [_vp])
_sig("rsl_quad3_velocities", ctypes.c_int, [_vp])
_sig("rsl_feq3", ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp])
_sig("rsl_moments3", ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp])

MOMENT3_FIELDS = ("N0", "N1", "N2", "N3", "T00", "T01", "T02", "T03", "T11", "T12", "T13", "T22", "T23", "T33",
                  "n", "E", "P", "T", "u0", "u1", "u2", "u3")


class Quadrature3:
    """Velocity set with Q_phi azimuths (rsl_make_quadrature3; owned library handle)."""

    def __init__(self, QL, Q, Qphi, NOm, T0=1.0):
        h = _vp()
        check(_lib.rsl_make_quadrature3(QL, Q, Qphi, NOm, float(T0), ctypes.byref(h)))
        self._h = h
        self.QL, self.Q, self.Qphi, self.NOm, self.T0 = QL, Q, Qphi, NOm, float(T0)
        self.V = _lib.rsl_quad3_velocities(h)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.rsl_free_quadrature3(h)
            self._h = None


def feq3(q3, state, dtype="f64", pitch=None, out=None, stream=None):
    """[V, pitch] equilibrium populations of the [ncell, 5] fp64 device states
    (n, T, u^x, u^y, u^z); rsl_feq3."""
    ncell = state.shape[0]
    pitch = ncell if pitch is None else pitch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if out is None:
        out = torch.zeros((q3.V, pitch), dtype=tdt, device=state.device)
    check(_lib.rsl_feq3(q3.handle, _p(state), ncell, C["RSL_F64"] if dtype == "f64" else C["RSL_F32"], _p(out),
                        pitch, _stream(stream)))
    return out


def moments3(q3, f, ncell, stream=None):
    """[ncell, RSL_NMOM3] moments and Landau frame of the [V, pitch] populations f; rsl_moments3."""
    out = torch.empty((ncell, C["RSL_NMOM3"]), dtype=torch.float64, device=f.device)
    dt = C["RSL_F64"] if f.dtype == torch.float64 else C["RSL_F32"]
    check(_lib.rsl_moments3(q3.handle, _p(f), dt, ncell, f.shape[1], _p(out), _stream(stream)))
    return out


# ------------------------------------------------------ in-loop feedback

_sig("rsl_mlp_inject", ctypes.c_int, [_vp, ctypes.POINTER(Problem), _vp, _vp, _vp])
_sig("rsl_project", ctypes.c_int, [_vp, ctypes.POINTER(Problem), _vp, _vp, ctypes.POINTER(Problem), _vp, _vp])


def inject(quad, problem, f_buf, y, stream=None):
    """Adds the population change that moves (T^00, T^0z, T^zz) by y * T^00
    ([nz, 3] fp32 device) to one Sod instance's f, in place; rsl_mlp_inject."""
    check(_lib.rsl_mlp_inject(quad.handle, ctypes.byref(problem), _p(f_buf), _p(y), _stream(stream)))


def project(q_hi, p_hi, f_hi, q_lo, p_lo, f_lo, stream=None):
    """f_lo <- the low-order state with f_hi's N^mu and T^{mu nu}; rsl_project."""
    check(_lib.rsl_project(q_hi.handle, ctypes.byref(p_hi), _p(f_hi), q_lo.handle, ctypes.byref(p_lo), _p(f_lo),
                           _stream(stream)))
