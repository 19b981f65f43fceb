"""Python binding of libse_mi355x.so (Spectral Ewald for Stokes flow, MI355X).

Argument marshalling only: every step of the computation runs in the HIP
library.  The ctypes entry points carry the C names of ``include/se.h``;
``Plan`` wraps them for torch device tensors (memory and streams only).
Importing this package fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libse_mi355x.so")

STOKESLET, ROTLET, STRESSLET, HARMONIC = 0, 1, 2, 3
KERNELS = {"stokeslet": STOKESLET, "rotlet": ROTLET, "stresslet": STRESSLET, "harmonic": HARMONIC}
TOL_REL, TOL_ABS = 0, 1
PREC_AUTO, PREC_FP64, PREC_FP32 = 0, 1, 2
SELECT_ANALYTIC, SELECT_LEARNED, SELECT_MANUAL = 0, 1, 2
POLLUTION_PAPER, POLLUTION_FINE = 0, 1
WINDOW_PKB, WINDOW_TG = 0, 1
WINDOWS = {"pkb": WINDOW_PKB, "tg": WINDOW_TG}

SE_OK = 0
SE_ERR_ARG, SE_ERR_UNSUPPORTED, SE_ERR_OUT_OF_BOX, SE_ERR_NONFINITE = -1, -2, -3, -4
SE_ERR_COINCIDENT, SE_ERR_TOL_UNREACHABLE, SE_ERR_NOMEM, SE_ERR_HIP, SE_ERR_STATE = -5, -6, -7, -8, -9
SE_ERR_SCRATCH = -10
MLP_NOALLOC_MAX_N = 16384
TILE_ITEMS_MAX = 16384  # largest gridding/gathering work item, in batches of 64 candidates
STATUS = {0: "SE_OK", -1: "SE_ERR_ARG", -2: "SE_ERR_UNSUPPORTED", -3: "SE_ERR_OUT_OF_BOX",
          -4: "SE_ERR_NONFINITE", -5: "SE_ERR_COINCIDENT", -6: "SE_ERR_TOL_UNREACHABLE",
          -7: "SE_ERR_NOMEM", -8: "SE_ERR_HIP", -9: "SE_ERR_STATE",
          -10: "SE_ERR_SCRATCH"}


class se_problem(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("periodicity", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("tol_kind", ctypes.c_int32),
                ("box", ctypes.c_double * 3), ("tol", ctypes.c_double),
                ("source_q", ctypes.c_double), ("xi", ctypes.c_double), ("n_rc", ctypes.c_double),
                ("safety", ctypes.c_double), ("precision", ctypes.c_int32),
                ("selector", ctypes.c_int32), ("n_src", ctypes.c_int64), ("n_tgt", ctypes.c_int64),
                ("targets_are_sources", ctypes.c_int32), ("n_rhs", ctypes.c_int32),
                ("device", ctypes.c_int32), ("pollution", ctypes.c_int32), ("window", ctypes.c_int32)]


class se_params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("P", ctypes.c_int32), ("nu_deg", ctypes.c_int32),
                ("f_M", ctypes.c_int32), ("M", ctypes.c_int32 * 3), ("n_fft", ctypes.c_int32 * 3),
                ("n0_fft", ctypes.c_int32 * 3), ("nstar_fft", ctypes.c_int32 * 3),
                ("kstar", ctypes.c_int32 * 2),
                ("xi", ctypes.c_double), ("rc", ctypes.c_double), ("beta", ctypes.c_double),
                ("h", ctypes.c_double * 3), ("L_ext", ctypes.c_double * 3), ("dL", ctypes.c_double * 3),
                ("R", ctypes.c_double), ("s0", ctypes.c_double), ("s_star", ctypes.c_double),
                ("tau_abs", ctypes.c_double), ("U", ctypes.c_double), ("est_real", ctypes.c_double),
                ("est_fourier", ctypes.c_double), ("est_window", ctypes.c_double),
                ("window", ctypes.c_int32), ("pad0", ctypes.c_int32), ("alpha", ctypes.c_double)]


EXPORTS = ["se_version", "se_status_string", "se_params_select", "se_plan_create", "se_plan_destroy",
           "se_plan_get_params", "se_plan_workspace_bytes", "se_plan_last_message", "se_set_geometry",
           "se_execute", "se_execute_split", "se_sync_status", "se_plan_set_timing", "se_plan_phase_times",
           "se_debug_cell_list", "se_plan_set_wrap", "se_plan_set_shape", "se_plan_get_shape", "se_batch_create", "se_batch_destroy",
           "se_batch_plan", "se_batch_set_geometry", "se_batch_execute", "se_batch_tune", "se_selector_features",
           "se_selector_train", "se_selector_save", "se_selector_load", "se_selector_ready", "se_selector_get",
           "se_selector_predict", "se_mlp_loss_grad", "se_mlp_loss_grad_noalloc", "se_mlp_forward", "se_mlp_adam", "se_ewald_reference", "se_bie_solve"]

PHASES = ["geometry", "strengths", "spread", "fft_fwd_xy", "fft_z_scale", "fft_inv_yx", "gather", "real_space",
          "epilogue"]


class se_train_cfg(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("device", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("seed", ctypes.c_uint64)]


MLP_IN, MLP_HID, MLP_OUT, MLP_NPARAM = 10, 64, 4, 5124
MLP_NORM = 2 * 10 + 2 * 4


class SEError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__("%s: %s" % (where, STATUS.get(status, str(status))))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libse_mi355x.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2210_01255_amd.build)")
    # One HIP runtime per process: torch's extension libraries ask for
    # libamdhip64.so and load the copy torch ships, whose soname is the
    # libamdhip64.so.7 this library links against.  Loading torch first makes
    # the library bind to that same copy, so that device pointers and streams
    # from torch are valid here; loaded the other way round the process would
    # hold two runtimes.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    P = ctypes.POINTER
    L.se_version.restype = i32
    L.se_version.argtypes = []
    L.se_status_string.restype = ctypes.c_char_p
    L.se_status_string.argtypes = [i32]
    L.se_params_select.restype = i32
    L.se_params_select.argtypes = [P(se_problem), P(se_params)]
    L.se_plan_create.restype = i32
    L.se_plan_create.argtypes = [P(se_problem), P(se_params), P(vp)]
    L.se_plan_destroy.restype = None
    L.se_plan_destroy.argtypes = [vp]
    L.se_plan_get_params.restype = i32
    L.se_plan_get_params.argtypes = [vp, P(se_params)]
    L.se_plan_workspace_bytes.restype = ctypes.c_size_t
    L.se_plan_workspace_bytes.argtypes = [vp]
    L.se_plan_last_message.restype = ctypes.c_char_p
    L.se_plan_last_message.argtypes = [vp]
    L.se_set_geometry.restype = i32
    L.se_set_geometry.argtypes = [vp, vp, vp, vp, vp]
    L.se_execute.restype = i32
    L.se_execute.argtypes = [vp, vp, vp, vp]
    L.se_execute_split.restype = i32
    L.se_execute_split.argtypes = [vp, vp, vp, vp, vp]
    L.se_sync_status.restype = i32
    L.se_sync_status.argtypes = [vp]
    L.se_plan_set_timing.restype = i32
    L.se_plan_set_timing.argtypes = [vp, i32]
    L.se_plan_phase_times.restype = i32
    L.se_plan_phase_times.argtypes = [vp, P(ctypes.c_double), P(i32), i32]
    L.se_debug_cell_list.restype = i32
    L.se_debug_cell_list.argtypes = [vp, i32, P(vp), P(vp), P(i32 * 3), P(i32 * 3)]
    L.se_plan_set_shape.restype = i32
    L.se_plan_set_shape.argtypes = [vp, i32, i32, i32]
    L.se_plan_get_shape.restype = i32
    L.se_plan_get_shape.argtypes = [vp, P(i32), P(i32), P(i32)]
    L.se_batch_create.restype = i32
    L.se_batch_create.argtypes = [P(se_problem), i32, P(vp)]
    L.se_batch_destroy.restype = i32
    L.se_batch_destroy.argtypes = [vp]
    L.se_batch_plan.restype = i32
    L.se_batch_plan.argtypes = [vp, i32, P(vp)]
    L.se_batch_set_geometry.restype = i32
    L.se_batch_set_geometry.argtypes = [vp, P(vp), P(vp), P(vp), vp]
    L.se_batch_execute.restype = i32
    L.se_batch_execute.argtypes = [vp, P(vp), P(vp), vp]
    L.se_batch_tune.restype = i32
    L.se_batch_tune.argtypes = [vp, P(vp), P(vp), vp]
    f32p = P(ctypes.c_float)
    L.se_selector_features.restype = i32
    L.se_selector_features.argtypes = [P(se_problem), f32p]
    L.se_selector_train.restype = i32
    L.se_selector_train.argtypes = [P(se_train_cfg), f32p, f32p, ctypes.c_int64, f32p]
    L.se_selector_save.restype = i32
    L.se_selector_save.argtypes = [ctypes.c_char_p]
    L.se_selector_load.restype = i32
    L.se_selector_load.argtypes = [ctypes.c_char_p]
    L.se_selector_ready.restype = i32
    L.se_selector_ready.argtypes = []
    L.se_selector_get.restype = i32
    L.se_selector_get.argtypes = [f32p, f32p]
    L.se_selector_predict.restype = i32
    L.se_selector_predict.argtypes = [vp, vp, ctypes.c_int64, vp]
    L.se_mlp_loss_grad.restype = i32
    L.se_mlp_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, vp]
    L.se_mlp_loss_grad_noalloc.restype = i32
    L.se_mlp_loss_grad_noalloc.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, vp]
    L.se_mlp_forward.restype = i32
    L.se_mlp_forward.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    L.se_ewald_reference.restype = i32
    L.se_ewald_reference.argtypes = [i32, i32, P(ctypes.c_double), ctypes.c_double, ctypes.c_int64, vp, vp, vp,
                                     ctypes.c_int64, vp, vp, i32, vp]
    L.se_bie_solve.restype = i32
    L.se_bie_solve.argtypes = [vp, ctypes.c_double, vp, vp, vp, i32, i32, ctypes.c_double, P(i32),
                               P(ctypes.c_double), vp]
    L.se_plan_set_wrap.restype = i32
    L.se_plan_set_wrap.argtypes = [vp, i32]
    L.se_mlp_adam.restype = i32
    L.se_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int64, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, vp]
    return L


lib = _load()

# Same names as the C ABI (thin forwards).
se_version = lib.se_version
se_status_string = lib.se_status_string
se_params_select = lib.se_params_select
se_plan_create = lib.se_plan_create
se_plan_destroy = lib.se_plan_destroy
se_plan_get_params = lib.se_plan_get_params
se_plan_workspace_bytes = lib.se_plan_workspace_bytes
se_plan_last_message = lib.se_plan_last_message
se_set_geometry = lib.se_set_geometry
se_execute = lib.se_execute
se_execute_split = lib.se_execute_split
se_sync_status = lib.se_sync_status
se_plan_set_timing = lib.se_plan_set_timing
se_plan_phase_times = lib.se_plan_phase_times
se_debug_cell_list = lib.se_debug_cell_list
se_plan_set_shape = lib.se_plan_set_shape
se_plan_get_shape = lib.se_plan_get_shape
se_batch_create = lib.se_batch_create
se_batch_destroy = lib.se_batch_destroy
se_batch_plan = lib.se_batch_plan
se_batch_set_geometry = lib.se_batch_set_geometry
se_batch_execute = lib.se_batch_execute
se_batch_tune = lib.se_batch_tune
se_selector_features = lib.se_selector_features
se_selector_train = lib.se_selector_train
se_selector_save = lib.se_selector_save
se_selector_load = lib.se_selector_load
se_selector_ready = lib.se_selector_ready
se_selector_get = lib.se_selector_get
se_selector_predict = lib.se_selector_predict
se_mlp_loss_grad = lib.se_mlp_loss_grad
se_mlp_loss_grad_noalloc = lib.se_mlp_loss_grad_noalloc
se_mlp_forward = lib.se_mlp_forward
se_mlp_adam = lib.se_mlp_adam
se_ewald_reference = lib.se_ewald_reference
se_bie_solve = lib.se_bie_solve


def make_problem(kernel="stokeslet", periodicity=3, box=(1.0, 1.0, 1.0), tol=1e-8, tol_kind=TOL_REL,
                 n_src=1, n_tgt=0, targets_are_sources=True, n_rhs=1, source_q=0.0, xi=0.0, n_rc=0.0,
                 safety=0.0, precision=PREC_FP64, selector=SELECT_ANALYTIC, device=0,
                 pollution=0, window=WINDOW_PKB) -> se_problem:
    p = se_problem()
    p.struct_size = ctypes.sizeof(se_problem)
    p.periodicity = int(periodicity)
    p.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    p.tol_kind = int(tol_kind)
    for i in range(3):
        p.box[i] = float(box[i])
    p.tol = float(tol)
    p.source_q = float(source_q)
    p.xi = float(xi)
    p.n_rc = float(n_rc)
    p.safety = float(safety)
    p.precision = int(precision)
    p.selector = int(selector)
    p.n_src = int(n_src)
    p.n_tgt = int(n_tgt)
    p.targets_are_sources = 1 if targets_are_sources else 0
    p.n_rhs = int(n_rhs)
    p.device = int(device)
    p.pollution = int(pollution)
    p.window = WINDOWS[window] if isinstance(window, str) else int(window)
    return p


def params_to_dict(par: se_params) -> dict:
    out = {}
    for name, _ in se_params._fields_:
        v = getattr(par, name)
        if hasattr(v, "__len__"):
            v = list(v)
        out[name] = v
    return out


def bie_solve(plan, alpha, weights, g, q0=None, restart=30, max_iter=300, tol=1e-10, stream=None):
    """GMRES for alpha q + D q = g (se_bie_solve) on a stresslet plan whose
    geometry (surface nodes and normals) is bound; g [n_rhs][n][3] (or
    [n][3]) device FP64.  Returns (q, iterations, relative residuals)."""
    import torch
    shp = (plan.n_rhs, plan.n_src, 3) if plan.n_rhs > 1 else (plan.n_src, 3)
    Plan._check(g, shp, "g")
    Plan._check(weights, (plan.n_src,), "weights")
    q = torch.zeros_like(g) if q0 is None else q0.clone()
    it = ctypes.c_int32(0)
    res = (ctypes.c_double * plan.n_rhs)()
    st = lib.se_bie_solve(plan.handle, ctypes.c_double(float(alpha)), _ptr(weights), _ptr(g), _ptr(q), int(restart),
                          int(max_iter), ctypes.c_double(float(tol)), ctypes.byref(it), res, _stream(stream))
    if st != SE_OK:
        raise SEError(st, "se_bie_solve")
    return q, int(it.value), list(res)


def ewald_reference(kernel, periodicity, box, x, strengths, normals=None, targets=None, xi=0.0, stream=None):
    """Direct Ewald sum on the GPU (se_ewald_reference): D = 3, 2, 1 or 0,
    device FP64 tensors [n][3]; returns u [n_tgt][3] on the same device."""
    import torch
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    Plan._check(x, (x.shape[0], 3), "src")
    Plan._check(strengths, (x.shape[0], 3), "strengths")
    Plan._check(normals, (x.shape[0], 3), "normals")
    nt = x.shape[0] if targets is None else targets.shape[0]
    if targets is not None:
        Plan._check(targets, (nt, 3), "targets")
    u = torch.empty((nt, 3), dtype=torch.float64, device=x.device)
    b = (ctypes.c_double * 3)(*[float(v) for v in box])
    st = lib.se_ewald_reference(int(kid), int(periodicity), b, ctypes.c_double(float(xi)), ctypes.c_int64(x.shape[0]),
                                _ptr(x), _ptr(strengths), _ptr(normals), ctypes.c_int64(nt), _ptr(targets), _ptr(u),
                                int(x.device.index or 0), _stream(stream))
    if st != SE_OK:
        raise SEError(st, "se_ewald_reference")
    return u


def select_params(**kw) -> dict:
    """Host-only parameter selection (se_params_select)."""
    prob = make_problem(**kw)
    par = se_params()
    st = lib.se_params_select(ctypes.byref(prob), ctypes.byref(par))
    if st != SE_OK:
        raise SEError(st, "se_params_select")
    return params_to_dict(par)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A plan bound to one device; tensors are torch float64 device tensors."""

    def __init__(self, manual: se_params | None = None, **kw):
        self.problem = make_problem(**kw)
        h = ctypes.c_void_p()
        st = lib.se_plan_create(ctypes.byref(self.problem),
                                ctypes.byref(manual) if manual is not None else None, ctypes.byref(h))
        if st != SE_OK:
            raise SEError(st, "se_plan_create")
        self._owned = True
        self._attach(h)

    def _attach(self, h):
        self.handle = h
        par = se_params()
        lib.se_plan_get_params(self.handle, ctypes.byref(par))
        self.params = params_to_dict(par)
        self.message = (lib.se_plan_last_message(self.handle) or b"").decode()
        self.kernel = self.problem.kernel
        self.n_src = self.problem.n_src
        self.n_tgt = self.problem.n_src if self.problem.targets_are_sources else self.problem.n_tgt
        self.n_rhs = self.problem.n_rhs

    @classmethod
    def _member(cls, handle, problem):
        """View of a plan owned by a Batch (not destroyed by close())."""
        self = cls.__new__(cls)
        self.problem = problem
        self._owned = False
        self._attach(handle)
        return self

    def close(self):
        if getattr(self, "handle", None):
            if getattr(self, "_owned", True):
                lib.se_plan_destroy(self.handle)
            self.handle = None

    def set_wrap(self, on=True):
        """Reduce periodic coordinates modulo L_i when binding (se_plan_set_wrap)."""
        st = lib.se_plan_set_wrap(self.handle, 1 if on else 0)
        if st != SE_OK:
            raise SEError(st, "se_plan_set_wrap")

    def set_shape(self, real_tb=0, fft_cols=0, tile_items=0):
        st = lib.se_plan_set_shape(self.handle, int(real_tb), int(fft_cols), int(tile_items))
        if st != SE_OK:
            raise SEError(st, "se_plan_set_shape")

    def get_shape(self):
        tb, fc, ti = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        st = lib.se_plan_get_shape(self.handle, ctypes.byref(tb), ctypes.byref(fc), ctypes.byref(ti))
        if st != SE_OK:
            raise SEError(st, "se_plan_get_shape")
        return tb.value, fc.value, ti.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _check(t, shape, name):
        import torch
        if t is None:
            return
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("%s must be a contiguous float64 device tensor" % name)
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), shape))

    def set_geometry(self, src, normals=None, targets=None, stream=None, check=False):
        self._check(src, (self.n_src, 3), "src")
        self._check(normals, (self.n_src, 3), "normals")
        if not self.problem.targets_are_sources:
            self._check(targets, (self.n_tgt, 3), "targets")
        self._keep = (src, normals, targets)
        st = lib.se_set_geometry(self.handle, _ptr(src), _ptr(normals), _ptr(targets), _stream(stream))
        if st != SE_OK:
            raise SEError(st, "se_set_geometry")
        if check:
            self.sync()

    def execute(self, strengths, out=None, stream=None):
        import torch
        shp = (self.n_rhs, self.n_src, 3) if self.n_rhs > 1 else (self.n_src, 3)
        self._check(strengths, shp, "strengths")
        if out is None:
            oshape = (self.n_rhs, self.n_tgt, 3) if self.n_rhs > 1 else (self.n_tgt, 3)
            out = torch.empty(oshape, dtype=torch.float64, device=strengths.device)
        st = lib.se_execute(self.handle, _ptr(strengths), _ptr(out), _stream(stream))
        if st != SE_OK:
            raise SEError(st, "se_execute")
        return out

    def execute_split(self, strengths, stream=None):
        import torch
        oshape = (self.n_rhs, self.n_tgt, 3) if self.n_rhs > 1 else (self.n_tgt, 3)
        ur = torch.empty(oshape, dtype=torch.float64, device=strengths.device)
        uf = torch.empty(oshape, dtype=torch.float64, device=strengths.device)
        st = lib.se_execute_split(self.handle, _ptr(strengths), _ptr(ur), _ptr(uf), _stream(stream))
        if st != SE_OK:
            raise SEError(st, "se_execute_split")
        return ur, uf

    def sync(self):
        st = lib.se_sync_status(self.handle)
        if st != SE_OK:
            raise SEError(st, "se_sync_status")

    def set_timing(self, on=True):
        st = lib.se_plan_set_timing(self.handle, 1 if on else 0)
        if st != SE_OK:
            raise SEError(st, "se_plan_set_timing")

    def phase_times(self):
        """{phase: (total ms, launches)} accumulated since set_timing(True)."""
        n = len(PHASES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int32 * n)()
        st = lib.se_plan_phase_times(self.handle, ms, cnt, n)
        if st != SE_OK:
            raise SEError(st, "se_plan_phase_times")
        return {PHASES[i]: (ms[i], cnt[i]) for i in range(n)}

    def cell_list(self, which=0):
        """(perm, cell_start, nbins_xyz, cell_width) as host numpy arrays."""
        import numpy as np
        import torch
        pp, cs = ctypes.c_void_p(), ctypes.c_void_p()
        nb, cw = (ctypes.c_int32 * 3)(), (ctypes.c_int32 * 3)()
        st = lib.se_debug_cell_list(self.handle, which, ctypes.byref(pp), ctypes.byref(cs),
                                    ctypes.byref(nb), ctypes.byref(cw))
        if st != SE_OK:
            raise SEError(st, "se_debug_cell_list")
        torch.cuda.synchronize()
        n = self.n_src if which == 0 else self.n_tgt
        nbins = nb[0] * nb[1] * nb[2]
        perm = np.empty(n, dtype=np.int32)
        start = np.empty(nbins + 1, dtype=np.int32)
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        hip.hipMemcpy(perm.ctypes.data, pp, perm.nbytes, 2)
        hip.hipMemcpy(start.ctypes.data, cs, start.nbytes, 2)
        return perm, start, list(nb), list(cw)


def _ptrs(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() if t is not None else 0 for t in ts])


class Batch:
    """Independent systems (uneven sizes, any periodicity) evaluated together.

    ``problems`` is a list of keyword dicts for make_problem.  On a non-default
    stream, the first execute with a given set of tensors runs eagerly and
    records a HIP graph that later calls with the same tensors replay.
    """

    def __init__(self, problems):
        n = len(problems)
        if n == 0:
            raise ValueError("empty batch")
        arr = (se_problem * n)(*[make_problem(**kw) for kw in problems])
        h = ctypes.c_void_p()
        st = lib.se_batch_create(arr, n, ctypes.byref(h))
        if st != SE_OK:
            raise SEError(st, "se_batch_create")
        self.handle = h
        self.plans = []
        for i in range(n):
            ph = ctypes.c_void_p()
            st = lib.se_batch_plan(self.handle, i, ctypes.byref(ph))
            if st != SE_OK:
                raise SEError(st, "se_batch_plan")
            self.plans.append(Plan._member(ph, arr[i]))

    def __len__(self):
        return len(self.plans)

    def close(self):
        if getattr(self, "handle", None):
            for p in self.plans:
                p.handle = None
            lib.se_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_geometry(self, srcs, normals=None, targets=None, stream=None):
        n = len(self.plans)
        normals = normals if normals is not None else [None] * n
        targets = targets if targets is not None else [None] * n
        for p, a, b, c in zip(self.plans, srcs, normals, targets):
            Plan._check(a, (p.n_src, 3), "src")
            Plan._check(b, (p.n_src, 3), "normals")
            if not p.problem.targets_are_sources:
                Plan._check(c, (p.n_tgt, 3), "targets")
        self._keep_geom = (list(srcs), list(normals), list(targets))
        st = lib.se_batch_set_geometry(self.handle, _ptrs(srcs), _ptrs(normals), _ptrs(targets), _stream(stream))
        if st != SE_OK:
            raise SEError(st, "se_batch_set_geometry")

    def _outs(self, strengths, outs):
        import torch
        if outs is None:
            outs = []
            for p, f in zip(self.plans, strengths):
                shp = (p.n_rhs, p.n_tgt, 3) if p.n_rhs > 1 else (p.n_tgt, 3)
                outs.append(torch.empty(shp, dtype=torch.float64, device=f.device))
        for p, f, o in zip(self.plans, strengths, outs):
            shp = (p.n_rhs, p.n_src, 3) if p.n_rhs > 1 else (p.n_src, 3)
            Plan._check(f, shp, "strengths")
            Plan._check(o, (p.n_rhs, p.n_tgt, 3) if p.n_rhs > 1 else (p.n_tgt, 3), "out")
        return outs

    def execute(self, strengths, outs=None, stream=None):
        if len(strengths) != len(self.plans):
            raise ValueError("one strengths tensor per system")
        outs = self._outs(strengths, outs)
        st = lib.se_batch_execute(self.handle, _ptrs(strengths), _ptrs(outs), _stream(stream))
        if st != SE_OK:
            raise SEError(st, "se_batch_execute")
        return outs

    def tune(self, strengths, outs=None, stream=None):
        """Autotune every member's launch shapes; returns [(real_tb, fft_cols, tile_items)]."""
        outs = self._outs(strengths, outs)
        st = lib.se_batch_tune(self.handle, _ptrs(strengths), _ptrs(outs), _stream(stream))
        if st != SE_OK:
            raise SEError(st, "se_batch_tune")
        return [p.get_shape() for p in self.plans]
