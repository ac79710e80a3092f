"""ctypes binding of libmdpe (include/mdpe.h), same entry-point names.

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of libmdpe.so.  There is no CPU fallback; loading fails loudly when
the library has not been built.

Device buffers are torch tensors (float64, contiguous, on the plan's
device); streams are torch.cuda streams (the current one by default).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdpe.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mdpe.h")

MDPE_OK, MDPE_EINVAL, MDPE_EUNSUPPORTED, MDPE_ENOMEM, MDPE_EDEVICE = 0, -1, -2, -3, -4
MDPE_KEEP_MONOMIAL_VALUES = 1
MDPE_COMPLEX = 2
MDPE_STREAM_OPERANDS = 4
MDPE_STAGE_OPERANDS = 8
MDPE_ASAP_LAYERS = 16
MDPE_FUSED_LAYERS = 32
MDPE_LAYER_LAUNCHES = 64
MDPE_CHAIN_LAUNCH = 128
MDPE_NO_CHAIN_LAUNCH = 256
MDPE_SINGLE_LAUNCH = 512
SUPPORTED_M = (1, 2, 3, 4, 5, 8, 10)


class MdpeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mdpe error {code}: {msg}")
        self.code = code


class PolyDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("N", ctypes.c_int32), ("d", ctypes.c_int32), ("m", ctypes.c_int32),
                ("nvars", ctypes.POINTER(ctypes.c_int32)), ("vars", ctypes.POINTER(ctypes.c_int32)),
                ("flags", ctypes.c_uint32), ("exps", ctypes.POINTER(ctypes.c_int32))]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_series", ctypes.c_int64), ("n_conv", ctypes.c_int64), ("n_add", ctypes.c_int64),
                ("n_layers", ctypes.c_int32), ("n_levels", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64),
                ("jobs_per_group", ctypes.c_int32), ("lane_steps", ctypes.c_int32),
                ("n", ctypes.c_int32), ("N", ctypes.c_int32), ("d", ctypes.c_int32), ("m", ctypes.c_int32),
                ("n_reverse", ctypes.c_int64), ("flags", ctypes.c_uint32), ("n_scale", ctypes.c_int64),
                ("waves_per_job", ctypes.c_int32), ("streamed", ctypes.c_int32),
                ("simple_dealing", ctypes.c_int32), ("balanced_layers", ctypes.c_int32),
                ("fused_components", ctypes.c_int32), ("fused_waves", ctypes.c_int32),
                ("chain_layers", ctypes.c_int32), ("chain_count", ctypes.c_int32), ("chain_waves", ctypes.c_int32),
                ("chain_window", ctypes.c_int32), ("chain_ring", ctypes.c_int32),
                ("single_launch", ctypes.c_int32), ("single_waves", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Times(ctypes.Structure):
    _fields_ = [("stage_ms", ctypes.c_double), ("cnv_ms", ctypes.c_double), ("add_ms", ctypes.c_double),
                ("gather_ms", ctypes.c_double), ("n_stage", ctypes.c_int64), ("n_cnv", ctypes.c_int64),
                ("n_add", ctypes.c_int64), ("n_gather", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchTile(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("d", ctypes.c_int32), ("jobs_per_group", ctypes.c_int32),
                ("groups_per_task", ctypes.c_int32), ("add_items_per_task", ctypes.c_int32),
                ("deal", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("n_tasks", ctypes.c_int64), ("n_conv_tasks", ctypes.c_int64),
                ("n_add_tasks", ctypes.c_int64), ("lds_bytes", ctypes.c_int64), ("grid", ctypes.c_int32),
                ("m1", ctypes.c_int32), ("m2", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_L = None


def lib():
    """Load libmdpe.so; raise if it is missing (no fallback)."""
    global _L
    if _L is not None:
        return _L
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    # torch first: its HIP runtime (torch/lib/libamdhip64.so, soname
    # libamdhip64.so.7) then satisfies the library's dependency, so both share
    # one runtime, one device context and one set of streams.  Loaded the
    # other way round, torch's libraries ask for the unversioned file name,
    # load a second runtime beside /opt/rocm's, and the library's HIP calls
    # then found no device.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.plan_polynomial.argtypes = [ctypes.POINTER(PolyDesc), ctypes.c_int, ctypes.POINTER(_vp)]
    L.plan_info.argtypes = [_vp, ctypes.POINTER(PlanInfo)]
    L.plan_layer_sizes.argtypes = [_vp, _i32p, _i32p]
    L.plan_conv_jobs.argtypes = [_vp, _i32p]
    L.plan_fused_jobs.argtypes = [_vp, _i32p]
    L.plan_chain_jobs.argtypes = [_vp, _i32p]
    L.chain_schedule.argtypes = [ctypes.c_int32] * 5 + [_i32p, ctypes.c_int64, _i32p, _i32p]
    L.check_chain_schedule.argtypes = [ctypes.c_int32] * 6 + [_i32p, ctypes.c_int32]
    L.plan_add_jobs.argtypes = [_vp, _i32p]
    L.plan_outputs.argtypes = [_vp, _i32p]
    L.plan_scale_jobs.argtypes = [_vp, _i32p]
    L.eval_and_diff.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.eval_and_diff_noalloc.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    L.eval_and_diff_profiled.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.profiler_create.argtypes = [ctypes.POINTER(_vp)]
    L.profiler_read.argtypes = [_vp, ctypes.POINTER(Times)]
    L.profiler_destroy.argtypes = [_vp]
    L.profiler_set_classes.argtypes = [_vp, ctypes.c_uint32]
    L.profiler_destroy.restype = None
    L.md_elementwise.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _vp, _vp, _vp, _vp]
    L.eval_adjoint.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.eval_adjoint_profiled.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.plan_reverse_jobs.argtypes = [_vp, _i32p]
    L.check_plan_jobs.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _i32p, ctypes.c_int64, _i32p,
                                  ctypes.c_int64, _i32p, _i32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
    L.plan_batch.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_char_p, ctypes.POINTER(_vp)]
    L.plan_batch_tiles.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(BatchTile), ctypes.c_int,
                                   ctypes.POINTER(_vp)]
    L.eval_and_diff_batch.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                      ctypes.POINTER(_vp), _vp, _vp]
    L.batch_info.argtypes = [_vp, ctypes.POINTER(BatchInfo)]
    L.batch_tasks.argtypes = [_vp, _i32p]
    L.batch_set_buffers.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                    ctypes.POINTER(_vp), ctypes.POINTER(_vp)]
    L.batch_launch.argtypes = [_vp, _vp]
    L.batch_launch_graph.argtypes = [_vp, _vp]
    L.batch_status.argtypes = [_vp]
    L.batch_set_grid.argtypes = [_vp, ctypes.c_int]
    L.batch_destroy.argtypes = [_vp]
    L.batch_destroy.restype = None
    L.plan_destroy.argtypes = [_vp]
    L.plan_destroy.restype = None
    L.last_error_string.argtypes = []
    L.last_error_string.restype = ctypes.c_char_p
    _L = L
    return L


def header_symbols(path: str = HEADER):
    """Function names declared in include/mdpe.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*(\w+)\s*\(", text, flags=re.M)))


def _check(rc):
    if rc != MDPE_OK:
        raise MdpeError(rc, lib().last_error_string().decode())
    return rc


def last_error_string() -> str:
    return lib().last_error_string().decode()


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream, device=None):
    if stream is None:
        import torch
        if device is not None:
            # the raw handle of torch's current stream on that device, without
            # building a Stream object
            return ctypes.c_void_p(torch._C._cuda_getCurrentRawStream(device))
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


class Plan:
    """A plan (plan_polynomial); device -1 builds a host-only plan for inspection."""

    def __init__(self, n, nvars, vars_, d, m, device=0, flags=0, exps=None):
        self.nvars = np.ascontiguousarray(nvars, dtype=np.int32)
        self.vars = np.ascontiguousarray(vars_, dtype=np.int32)
        self.exps = None if exps is None else np.ascontiguousarray(exps, dtype=np.int32)
        if self.exps is not None and self.exps.shape != self.vars.shape:
            raise ValueError("exps must have one exponent per entry of vars")
        desc = PolyDesc(int(n), int(self.nvars.shape[0]), int(d), int(m),
                        self.nvars.ctypes.data_as(_i32p), self.vars.ctypes.data_as(_i32p), int(flags),
                        self.exps.ctypes.data_as(_i32p) if self.exps is not None else None)
        h = _vp()
        _check(lib().plan_polynomial(ctypes.byref(desc), int(device), ctypes.byref(h)))
        self._h = h
        self.device = device
        info = PlanInfo()
        _check(lib().plan_info(h, ctypes.byref(info)))
        self.info = info.as_dict()

    @classmethod
    def for_workload(cls, w, device=0, flags=0):
        if getattr(w, "cx", False):
            flags |= MDPE_COMPLEX
        return cls(w.n, w.nvars, w.vars, w.d, w.m, device, flags, getattr(w, "exps", None))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _L is not None:
            _L.plan_destroy(h)
            self._h = None

    def reverse_jobs(self):
        rows = np.zeros((max(self.info["n_reverse"], 1), 3), dtype=np.int32)
        _check(lib().plan_reverse_jobs(self._h, rows.ctypes.data_as(_i32p)))
        return rows[: self.info["n_reverse"]]

    @property
    def handle(self):
        return self._h

    def layer_sizes(self):
        conv = np.zeros(max(self.info["n_layers"], 1), dtype=np.int32)
        add = np.zeros(max(self.info["n_levels"], 1), dtype=np.int32)
        _check(lib().plan_layer_sizes(self._h, conv.ctypes.data_as(_i32p), add.ctypes.data_as(_i32p)))
        return list(conv[: self.info["n_layers"]]), list(add[: self.info["n_levels"]])

    def conv_jobs(self):
        rows = np.zeros((max(self.info["n_conv"], 1), 4), dtype=np.int32)
        _check(lib().plan_conv_jobs(self._h, rows.ctypes.data_as(_i32p)))
        return rows[: self.info["n_conv"]]

    def fused_jobs(self):
        """MDPE_FUSED_LAYERS plans: rows {component, layer, t1, t2, t3} in fused launch order."""
        rows = np.zeros((max(self.info["n_conv"], 1), 5), dtype=np.int32)
        _check(lib().plan_fused_jobs(self._h, rows.ctypes.data_as(_i32p)))
        return rows[: self.info["n_conv"]]

    def chain_jobs(self):
        """MDPE_CHAIN_LAUNCH plans: rows {chain, position, t1, t2, t3}, chain after chain."""
        n = int(sum(self.layer_sizes()[0][: self.info["chain_layers"]]))
        rows = np.zeros((max(n, 1), 5), dtype=np.int32)
        _check(lib().plan_chain_jobs(self._h, rows.ctypes.data_as(_i32p)))
        return rows[:n]

    def add_jobs(self):
        rows = np.zeros((max(self.info["n_add"], 1), 3), dtype=np.int32)
        _check(lib().plan_add_jobs(self._h, rows.ctypes.data_as(_i32p)))
        return rows[: self.info["n_add"]]

    def outputs(self):
        out = np.zeros(1 + self.info["n"], dtype=np.int32)
        _check(lib().plan_outputs(self._h, out.ctypes.data_as(_i32p)))
        return out

    def scale_jobs(self):
        rows = np.zeros((max(self.info["n_scale"], 1), 3), dtype=np.int32)
        _check(lib().plan_scale_jobs(self._h, rows.ctypes.data_as(_i32p)))
        return rows[: self.info["n_scale"]]


def check_plan_jobs(n, N, n_series, conv_rows, add_rows, out_slots=None, extra_staged=None, waves_per_job=1,
                    streamed=False):
    """Host-only check of job rows ({layer, t1, t2, t3} and {level, t1, t2}, as
    Plan.conv_jobs / Plan.add_jobs return them); raises MdpeError naming the
    violated rule."""
    conv = np.ascontiguousarray(np.asarray(conv_rows, dtype=np.int32).reshape(-1, 4))
    add = np.ascontiguousarray(np.asarray(add_rows, dtype=np.int32).reshape(-1, 3))
    out = None if out_slots is None else np.ascontiguousarray(out_slots, dtype=np.int32)
    if out is not None and out.shape != (int(n) + 1,):
        raise ValueError("out_slots must have 1 + n entries")
    extra = np.ascontiguousarray(np.zeros(0) if extra_staged is None else extra_staged, dtype=np.int32)
    _check(lib().check_plan_jobs(int(n), int(N), int(n_series), conv.ctypes.data_as(_i32p), int(conv.shape[0]),
                                 add.ctypes.data_as(_i32p), int(add.shape[0]),
                                 out.ctypes.data_as(_i32p) if out is not None else None,
                                 extra.ctypes.data_as(_i32p) if extra.size else None, int(extra.size),
                                 int(waves_per_job), int(bool(streamed))))


def chain_schedule(L, d, waves, window, ring):
    """Host-only lane schedule of one chain: (codes int32[64*waves][stride], steps)."""
    stride, steps = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().chain_schedule(int(L), int(d), int(waves), int(window), int(ring), None, 0, ctypes.byref(stride),
                                ctypes.byref(steps)))
    codes = np.zeros((64 * int(waves), stride.value), dtype=np.int32)
    _check(lib().chain_schedule(int(L), int(d), int(waves), int(window), int(ring), codes.ctypes.data_as(_i32p),
                                int(codes.size), ctypes.byref(stride), ctypes.byref(steps)))
    return codes, steps.value


def check_chain_schedule(L, d, waves, window, ring, steps, codes):
    """Raise MdpeError unless `codes` meets the chain kernel's ordering rules."""
    codes = np.ascontiguousarray(codes, dtype=np.int32)
    _check(lib().check_chain_schedule(int(L), int(d), int(waves), int(window), int(ring), int(steps),
                                      codes.ctypes.data_as(_i32p), int(codes.shape[1])))


def plan_polynomial(n, nvars, vars_, d, m, device=0) -> Plan:
    return Plan(n, nvars, vars_, d, m, device)


def eval_and_diff(plan: Plan, coeff, z, value, grad, workspace, stream=None, device=None):
    """Enqueue one evaluation on `stream` (tensors on the plan's device)."""
    _check(lib().eval_and_diff(plan.handle, _ptr(coeff), _ptr(z), _ptr(value), _ptr(grad), _ptr(workspace),
                               _stream(stream, device)))


def eval_and_diff_noalloc(plan: Plan, coeff, z, value, grad, stream=None):
    """Enqueue one evaluation on `stream` over the library's fixed workspace."""
    _check(lib().eval_and_diff_noalloc(plan.handle, _ptr(coeff), _ptr(z), _ptr(value), _ptr(grad),
                                       _stream(stream)))


MDPE_TIME_STAGE, MDPE_TIME_CONV, MDPE_TIME_ADD, MDPE_TIME_GATHER = 1, 2, 4, 8


class Profiler:
    """HIP-event timing of the launches of eval_and_diff / eval_adjoint.
    classes: mask of MDPE_TIME_* (None: all launches)."""

    def __init__(self, classes=None):
        h = _vp()
        _check(lib().profiler_create(ctypes.byref(h)))
        self._h = h
        if classes is not None:
            _check(lib().profiler_set_classes(h, int(classes)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _L is not None:
            _L.profiler_destroy(h)
            self._h = None

    def read(self) -> dict:
        t = Times()
        _check(lib().profiler_read(self._h, ctypes.byref(t)))
        return t.as_dict()


def eval_and_diff_profiled(plan: Plan, coeff, z, value, grad, workspace, prof: Profiler, stream=None):
    _check(lib().eval_and_diff_profiled(plan.handle, _ptr(coeff), _ptr(z), _ptr(value), _ptr(grad),
                                        _ptr(workspace), _stream(stream), prof._h))


def eval_adjoint(plan: Plan, ybar, workspace, grad, coeff_bar, z_bar, stream=None, profiler=None):
    """Enqueue the reverse pass (plan built with MDPE_KEEP_MONOMIAL_VALUES):
    workspace and grad from the preceding eval_and_diff."""
    if profiler is None:
        _check(lib().eval_adjoint(plan.handle, _ptr(ybar), _ptr(workspace), _ptr(grad), _ptr(coeff_bar),
                                  _ptr(z_bar), _stream(stream)))
    else:
        _check(lib().eval_adjoint_profiled(plan.handle, _ptr(ybar), _ptr(workspace), _ptr(grad), _ptr(coeff_bar),
                                           _ptr(z_bar), _stream(stream), profiler._h))


def md_elementwise(op, x, y, z, stream=None):
    """z = x op y on float64 device tensors: op 'add' or 'mul' on planar [m][count],
    'cadd' or 'cmul' on complex [2][m][count] (real limbs, then imaginary limbs)."""
    code = {"add": 0, "mul": 1, "cadd": 2, "cmul": 3}[op]
    if x.dim() != (3 if code >= 2 else 2) or x.shape[0] != (2 if code >= 2 else x.shape[0]):
        raise ValueError(f"{op}: bad operand shape {tuple(x.shape)}")
    m, count = x.shape[-2], x.shape[-1]
    for t in (x, y, z):
        if t.shape != x.shape or not t.is_contiguous():
            raise ValueError("x, y, z must be contiguous tensors of one shape")
    _check(lib().md_elementwise(code, int(m), int(count), _ptr(x), _ptr(y), _ptr(z), _stream(stream)))


class Polynomial:
    """Plan + workspace + output buffers on one device: the convenience API.

    >>> P = Polynomial(n, nvars, vars, d, m)
    >>> value, grad = P.eval_and_diff(coeff, z)   # float64 tensors [m][N+1][d+1], [m][n][d+1]

    complex=True: complex series, every tensor with a leading axis of two
    (real parts, then imaginary parts), e.g. coeff [2][m][N+1][d+1].
    exps: one exponent per entry of vars_ (None: every exponent one).
    keep_monomials: keep each monomial's product of variables for adjoint().
    stream_operands / fused_layers: None lets the plan choose; True / False
    forces operands read from global memory (else staged in LDS) / every
    convolution layer in one launch (else one launch per layer).
    chain_launch: True forces the chains of products into one pipelined
    launch (MDPE_CHAIN_LAUNCH), False excludes it (MDPE_NO_CHAIN_LAUNCH), None
    lets the plan choose; fused_layers=False excludes it too.
    single_launch: True forces the whole evaluation into one workgroup's
    launch (MDPE_SINGLE_LAUNCH; plans choose it by themselves when tiny).
    asap_layers: every convolution at its earliest layer (no balancing).
    """

    def __init__(self, n, nvars, vars_, d, m, device=None, keep_monomials=False, complex=False, exps=None,
                 stream_operands=None, asap_layers=False, fused_layers=None, alloc_workspace=True,
                 chain_launch=None, single_launch=False):
        import torch
        if device is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = torch.device(device)
        # stream_operands: None lets the plan choose, True / False forces it
        flags = ((MDPE_KEEP_MONOMIAL_VALUES if keep_monomials else 0) | (MDPE_COMPLEX if complex else 0) |
                 (MDPE_STREAM_OPERANDS if stream_operands is True else 0) |
                 (MDPE_STAGE_OPERANDS if stream_operands is False else 0) |
                 (MDPE_ASAP_LAYERS if asap_layers else 0) |
                 # fused_layers: None lets the plan choose, True / False forces it
                 (MDPE_FUSED_LAYERS if fused_layers is True else 0) |
                 (MDPE_LAYER_LAUNCHES if fused_layers is False else 0) |
                 (MDPE_CHAIN_LAUNCH if chain_launch is True else 0) |
                 (MDPE_NO_CHAIN_LAUNCH if chain_launch is False else 0) |
                 (MDPE_SINGLE_LAUNCH if single_launch else 0))
        self.plan = Plan(n, nvars, vars_, d, m, self.device.index or 0, flags, exps)
        self.n, self.N, self.d, self.m = int(n), int(self.plan.info["N"]), int(d), int(m)
        self.complex = bool(complex)
        self._lead = (2, self.m) if complex else (self.m,)
        nbytes = int(self.plan.info["workspace_bytes"])
        # 256-byte aligned by the caching allocator; alloc_workspace=False
        # leaves it to the caller (a view of a batch's shared workspace)
        self.workspace = (torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=self.device)
                          if alloc_workspace else None)

    @classmethod
    def for_workload(cls, w, device=None, keep_monomials=False, stream_operands=None, asap_layers=False,
                     fused_layers=None, alloc_workspace=True, chain_launch=None, single_launch=False):
        return cls(w.n, w.nvars, w.vars, w.d, w.m, device, keep_monomials, getattr(w, "cx", False),
                   getattr(w, "exps", None), stream_operands, asap_layers, fused_layers, alloc_workspace,
                   chain_launch, single_launch)

    def new_workspace(self):
        import torch
        return torch.empty_like(self.workspace)

    def adjoint(self, ybar, grad, workspace=None, stream=None, profiler=None):
        """Reverse pass after eval_and_diff on `workspace` (default: this
        object's), with the gradient `grad` that call returned."""
        import torch
        if ybar.dtype != torch.float64 or tuple(ybar.shape) != (self.m, self.d + 1) or not ybar.is_contiguous():
            raise ValueError(f"ybar: need a contiguous float64 tensor of shape {(self.m, self.d + 1)}")
        gshape = (self.m, self.n, self.d + 1)
        if grad.dtype != torch.float64 or tuple(grad.shape) != gshape or not grad.is_contiguous():
            raise ValueError(f"grad: need a contiguous float64 tensor of shape {gshape}")
        cbar = torch.empty((self.m, self.N + 1, self.d + 1), dtype=torch.float64, device=self.device)
        zbar = torch.empty((self.m, self.n, self.d + 1), dtype=torch.float64, device=self.device)
        eval_adjoint(self.plan, ybar, self.workspace if workspace is None else workspace, grad, cbar, zbar, stream,
                     profiler)
        return cbar, zbar

    def _check_inputs(self, coeff, z):
        import torch
        for name, t, shape in (("coeff", coeff, self._lead + (self.N + 1, self.d + 1)),
                               ("z", z, self._lead + (self.n, self.d + 1))):
            if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != shape or t.device != self.device:
                raise ValueError(f"{name}: need a contiguous float64 tensor of shape {shape} on {self.device}")

    def eval_and_diff(self, coeff, z, value=None, grad=None, stream=None, profiler=None, workspace=None):
        import torch
        ws = self.workspace if workspace is None else workspace
        if value is None:
            value = torch.empty(self._lead + (self.d + 1,), dtype=torch.float64, device=self.device)
        if grad is None:
            grad = torch.empty(self._lead + (self.n, self.d + 1), dtype=torch.float64, device=self.device)
        # the tensors of the previous call, checked then: repeated calls on the
        # same buffers (a serving loop) skip the checks; their sizes are fixed
        # by the plan, and a tensor's storage pointer is compared every call
        key = (coeff.data_ptr(), z.data_ptr(), value.data_ptr(), grad.data_ptr())
        last = getattr(self, "_checked", None)
        if (last is None or last[0] is not coeff or last[1] is not z or last[2] is not value or last[3] is not grad
                or self._checked_ptrs != key):
            self._check_inputs(coeff, z)
            for name, t, shape in (("value", value, self._lead + (self.d + 1,)),
                                   ("grad", grad, self._lead + (self.n, self.d + 1))):
                if (t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != shape
                        or t.device != self.device):
                    raise ValueError(f"{name}: need a contiguous float64 tensor of shape {shape} on {self.device}")
            self._checked, self._checked_ptrs = (coeff, z, value, grad), key
        if profiler is None:
            eval_and_diff(self.plan, coeff, z, value, grad, ws, stream, self.device.index or 0)
        else:
            eval_and_diff_profiled(self.plan, coeff, z, value, grad, ws, profiler, stream)
        return value, grad


TUNE_CACHE = os.path.join(_HERE, "tune_cache.json")


class Batch:
    """plan_batch over Plan objects (kept alive by the batch).

    tune_cache: path of the autotuner's cache (plan_batch reads it); else
    tiles: optional list of dicts {m, d, jobs_per_group, groups_per_task,
    add_items_per_task} (zero / missing fields take the defaults),
    passed to plan_batch_tiles.
    """

    def __init__(self, plans, tiles=None, tune_cache=None):
        self.plans = list(plans)
        arr = (_vp * len(self.plans))(*[p.handle.value for p in self.plans])
        h = _vp()
        if tune_cache is not None:
            if tiles is not None:
                raise ValueError("give tiles or tune_cache, not both")
            _check(lib().plan_batch(arr, len(self.plans), os.fsencode(tune_cache), ctypes.byref(h)))
        else:
            tl = list(tiles or [])
            tarr = (BatchTile * max(len(tl), 1))()
            for q, t in enumerate(tl):
                tarr[q] = BatchTile(int(t["m"]), int(t["d"]), int(t.get("jobs_per_group", 0)),
                                    int(t.get("groups_per_task", 0)), int(t.get("add_items_per_task", 0)),
                                    int(t.get("deal", 0)))
            _check(lib().plan_batch_tiles(arr, len(self.plans), tarr, len(tl), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _L is not None:
            _L.batch_destroy(h)
            self._h = None

    def info(self):
        i = BatchInfo()
        _check(lib().batch_info(self._h, ctypes.byref(i)))
        return i.as_dict()

    def tasks(self):
        n = self.info()["n_tasks"]
        rows = np.zeros((max(n, 1), 6), dtype=np.int32)
        _check(lib().batch_tasks(self._h, rows.ctypes.data_as(_i32p)))
        return rows[:n]

    def set_buffers(self, coeffs, zs, values, grads, workspaces):
        def arr(ts):
            return (_vp * len(ts))(*[t.data_ptr() for t in ts])
        self._keep = (coeffs, zs, values, grads, workspaces)
        _check(lib().batch_set_buffers(self._h, arr(coeffs), arr(zs), arr(values), arr(grads), arr(workspaces)))

    def eval_and_diff(self, coeffs, zs, values, grads, workspace, stream=None):
        """eval_and_diff_batch: one graph replay on `stream`, rebinding the
        pointer table on the stream when a buffer changed."""
        def arr(ts):
            return (_vp * len(ts))(*[t.data_ptr() for t in ts])
        self._keep_eval = (coeffs, zs, values, grads, workspace)
        _check(lib().eval_and_diff_batch(self._h, arr(coeffs), arr(zs), arr(values), arr(grads), _ptr(workspace),
                                         _stream(stream)))

    def launch(self, stream=None):
        _check(lib().batch_launch(self._h, _stream(stream)))

    def launch_graph(self, stream=None):
        _check(lib().batch_launch_graph(self._h, _stream(stream)))

    def status(self):
        _check(lib().batch_status(self._h))

    def set_grid(self, grid):
        _check(lib().batch_set_grid(self._h, int(grid)))


class BatchedPolynomials:
    """Polynomials (one Polynomial each, with its plan) run as one batch.

    The instances share one workspace of batch_info().workspace_bytes; each
    Polynomial's workspace is its part of it, so the instances can also be
    evaluated one by one (Polynomial.eval_and_diff) on the same memory.
    tune_cache: the autotuner's cache, read by plan_batch; else tiles (a list
    of tile dicts, plan_batch_tiles)."""

    def __init__(self, workloads, device=None, tiles=None, tune_cache=None):
        import torch
        if device is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = torch.device(device)
        self.polys = [Polynomial.for_workload(w, self.device, alloc_workspace=False) for w in workloads]
        self._tiles, self._tune_cache = tiles, tune_cache
        self.batch = Batch([P.plan for P in self.polys], tiles, tune_cache)
        total = int(self.batch.info()["workspace_bytes"])
        self.workspace = torch.empty(max(total // 8, 1), dtype=torch.float64, device=self.device)
        off = 0
        for P in self.polys:
            nb = int(P.plan.info["workspace_bytes"])
            P.workspace = self.workspace[off // 8: off // 8 + max(nb // 8, 1)]
            off += (nb + 255) // 256 * 256
        if off != total:
            raise RuntimeError(f"batch workspace layout: {off} bytes against {total}")
        self.values = [torch.empty((P.m, P.d + 1), dtype=torch.float64, device=self.device) for P in self.polys]
        self.grads = [torch.empty((P.m, P.n, P.d + 1), dtype=torch.float64, device=self.device) for P in self.polys]

    def bind(self, coeffs, zs):
        for P, c, z in zip(self.polys, coeffs, zs):
            P._check_inputs(c, z)
        self._inputs = (coeffs, zs)
        self.batch.set_buffers(coeffs, zs, self.values, self.grads, [P.workspace for P in self.polys])

    def eval_and_diff(self, coeffs, zs, stream=None):
        """All instances in one graph replay (eval_and_diff_batch); returns the
        per-instance value and gradient tensors."""
        for P, c, z in zip(self.polys, coeffs, zs):
            P._check_inputs(c, z)
        self.batch.eval_and_diff(coeffs, zs, self.values, self.grads, self.workspace, stream)
        return self.values, self.grads

    def set_tiles(self, tiles):
        """Rebuild the task queue with other tiles (plans and buffers are kept)."""
        self.batch = Batch([P.plan for P in self.polys], tiles)
        if getattr(self, "_inputs", None) is not None:
            self.bind(*self._inputs)

    def run(self, graph=False, stream=None):
        (self.batch.launch_graph if graph else self.batch.launch)(stream)
        return self.values, self.grads
