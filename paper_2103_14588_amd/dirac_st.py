"""Python binding of the C ABI in include/dirac_st.h (ctypes).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the solve runs in libdirac_st.so.  Importing
this module fails loudly if the library has not been built
(``python -m paper_2103_14588_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdirac_st.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libdirac_st.so is not built; run `python -m paper_2103_14588_amd.build`")
_lib = C.CDLL(LIB_PATH)

OK, NOT_CONVERGED, EINVAL, EHIP, EBREAKDOWN, ENOSPACE = 0, 1, -1, -2, -3, -4
V_NONE, V_STEP, V_SMOOTH = 0, 1, 2
PC_NONE, PC_BLOCK_JACOBI, PC_SPECTRAL, PC_LINE, PC_TIME_SLABS = 0, 1, 2, 3, 4
PC_NAMES = {"none": PC_NONE, "bj": PC_BLOCK_JACOBI, "spectral": PC_SPECTRAL, "line": PC_LINE,
            "slabs": PC_TIME_SLABS}


class Problem(C.Structure):
    _fields_ = [("d", C.c_int32), ("nc", C.c_int32), ("n", C.c_int32 * 4), ("len", C.c_double * 4),
                ("m", C.c_double), ("vkind", C.c_int32), ("v0", C.c_double), ("x0", C.c_double),
                ("lw", C.c_double)]


class BSR(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val64", C.c_void_p),
                ("val32", C.c_void_p), ("bjinv64", C.c_void_p), ("bjinv32", C.c_void_p),
                ("nrows", C.c_int64), ("nnzb", C.c_int64), ("nc", C.c_int32),
                ("singular_blocks", C.c_int32), ("prob", Problem)]


class Opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_it", C.c_int32), ("pc", C.c_int32),
                ("precision", C.c_int32), ("max_cycles", C.c_int32), ("rtol", C.c_double),
                ("inner_rtol", C.c_double), ("vbar", C.c_double), ("time_slabs", C.c_int32),
                ("matrix_free", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("cycles", C.c_int32), ("converged", C.c_int32),
                ("singular_blocks", C.c_int32), ("relres", C.c_double), ("est", C.c_double),
                ("ms", C.c_double), ("history", C.POINTER(C.c_double)), ("history_len", C.c_int32),
                ("fallback", C.c_int32)]


class NNStruct(C.Structure):
    _fields_ = [("params", C.c_void_p), ("adam_m", C.c_void_p), ("adam_v", C.c_void_p),
                ("w16", C.c_void_p), ("wt16", C.c_void_p), ("step", C.c_int32), ("out_gain", C.c_float)]


_vp, _i32, _i64 = C.c_void_p, C.c_int32, C.c_int64
_lib.dirac_st_last_error.restype = C.c_char_p
_lib.dirac_st_sizes.argtypes = [C.POINTER(Problem), C.POINTER(_i64), C.POINTER(_i64)]
_lib.dirac_st_assemble.argtypes = [C.POINTER(Problem), _vp, C.POINTER(BSR), _vp, _vp]
_lib.dirac_st_spmv.argtypes = [C.POINTER(BSR), _i32, _vp, _vp, _vp]
_lib.dirac_st_pc_apply.argtypes = [C.POINTER(BSR), C.POINTER(Opts), _vp, _vp, _vp, C.c_size_t, _vp]
_lib.dirac_st_workspace_bytes.argtypes = [C.POINTER(BSR), C.POINTER(Opts), _i32]
_lib.dirac_st_workspace_bytes.restype = C.c_size_t
_lib.dirac_st_gmres.argtypes = [C.POINTER(BSR), _vp, _vp, C.POINTER(Opts), _vp, C.c_size_t,
                                C.POINTER(Stats), _vp]

_lib.dirac_st_nn_param_count.restype = C.c_size_t
_lib.dirac_st_spmv_mf.argtypes = [C.POINTER(Problem), _i32, _vp, _vp, _vp]
_lib.dirac_st_rhs_mf.argtypes = [C.POINTER(Problem), _vp, _vp, _vp]
_lib.dirac_st_slice_moments.argtypes = [C.POINTER(Problem), _vp, _vp, C.c_double, _vp, _vp]
_lib.dirac_st_bicgstab_workspace_bytes.argtypes = [C.POINTER(BSR), C.POINTER(Opts)]
_lib.dirac_st_bicgstab_workspace_bytes.restype = C.c_size_t
_lib.dirac_st_bicgstab.argtypes = [C.POINTER(BSR), _vp, _vp, C.POINTER(Opts), _vp, C.c_size_t,
                                   C.POINTER(Stats), _vp]
_lib.dirac_st_nn_workspace_bytes.argtypes = [_i32, _i32, _i32, _i32]
_lib.dirac_st_nn_workspace_bytes.restype = C.c_size_t
_lib.dirac_st_nn_pack.argtypes = [C.POINTER(NNStruct), _vp]
_lib.dirac_st_nn_forward.argtypes = [C.POINTER(NNStruct), _i32, _i32, _i32, _vp, C.c_double, _vp, _vp,
                                     C.c_size_t, _vp]
_lib.dirac_st_nn_backward.argtypes = [C.POINTER(NNStruct), _i32, _i32, _i32, _vp, C.c_double, _vp, _vp,
                                      _vp, C.c_size_t, _vp]
_lib.dirac_st_nn_train_step.argtypes = [C.POINTER(NNStruct), _i32, _i32, _i32, _vp, _vp, C.c_float, _vp,
                                        _vp, C.c_size_t, _vp]
_lib.dirac_st_fgmres_nn.argtypes = [C.POINTER(BSR), _vp, _vp, C.POINTER(NNStruct), C.POINTER(Opts), _vp,
                                    C.c_size_t, C.POINTER(Stats), _vp]

_BSRP = C.POINTER(BSR)
_lib.dirac_st_batched_workspace_bytes.argtypes = [_i32, C.POINTER(_BSRP), C.POINTER(Opts)]
_lib.dirac_st_batched_workspace_bytes.restype = C.c_size_t
_lib.dirac_st_fgmres_batched.argtypes = [_i32, C.POINTER(_BSRP), C.POINTER(_vp), C.POINTER(_vp),
                                         C.POINTER(Opts), _vp, C.c_size_t, C.POINTER(Stats), _vp]
_lib.dirac_st_spmv_batched_workspace_bytes.argtypes = [_i32, C.POINTER(_BSRP)]
_lib.dirac_st_spmv_batched_workspace_bytes.restype = C.c_size_t
_lib.dirac_st_spmv_batched.argtypes = [_i32, C.POINTER(_BSRP), _i32, C.POINTER(_vp), C.POINTER(_vp), _i32,
                                       _vp, C.c_size_t, _vp]
_lib.dirac_st_time_eigen.argtypes = [_i32, C.c_double, _vp, _vp, _vp]
_lib.dirac_st_timing.argtypes = [_i32]
_lib.dirac_st_timing_read.argtypes = [_i32, C.POINTER(_i64), C.POINTER(C.c_double)]
_lib.dirac_st_batched_set_lanes.argtypes = [_i32, _i32, _i32]
_lib.dirac_st_batched_lanes.argtypes = [_i32, _i32, _i64]
_lib.dirac_st_batched_lanes.restype = _i32

EXPORTS = ["dirac_st_last_error", "dirac_st_sizes", "dirac_st_assemble", "dirac_st_spmv",
           "dirac_st_pc_apply", "dirac_st_workspace_bytes", "dirac_st_gmres",
           "dirac_st_nn_param_count", "dirac_st_nn_workspace_bytes", "dirac_st_nn_pack",
           "dirac_st_nn_forward", "dirac_st_nn_backward", "dirac_st_nn_train_step",
           "dirac_st_fgmres_nn", "dirac_st_batched_workspace_bytes", "dirac_st_fgmres_batched",
           "dirac_st_spmv_batched_workspace_bytes", "dirac_st_spmv_batched",
           "dirac_st_batched_set_lanes", "dirac_st_batched_lanes", "dirac_st_time_eigen",
           "dirac_st_timing", "dirac_st_timing_read", "dirac_st_bicgstab_workspace_bytes",
           "dirac_st_bicgstab", "dirac_st_spmv_mf", "dirac_st_rhs_mf",
           "dirac_st_slice_moments"]


class DiracError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("dirac_st error %d: %s" % (code, msg))
        self.code = code


def last_error() -> str:
    return _lib.dirac_st_last_error().decode()


def _check(rc, allow=(OK,)):
    if rc not in allow:
        raise DiracError(rc, last_error())
    return rc


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def make_problem(spec) -> Problem:
    """From paper_2103_14588_amd.inputs.Spec (or any object with the same fields)."""
    p = Problem()
    p.d, p.nc = spec.d, spec.nc
    for a in range(4):
        p.n[a] = spec.n[a] if a <= spec.d else 1
        p.len[a] = spec.lens[a] if a <= spec.d else 1.0
    p.m, p.vkind, p.v0, p.x0, p.lw = spec.m, spec.vkind, spec.v0, spec.x0, spec.lw
    return p


def sizes(spec):
    p = make_problem(spec)
    nr, nb = _i64(), _i64()
    _check(_lib.dirac_st_sizes(C.byref(p), C.byref(nr), C.byref(nb)))
    return nr.value, nb.value


@dataclass
class Operator:
    """Assembled operator; owns its device tensors."""
    spec: object
    bsr: BSR
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val64: torch.Tensor
    val32: torch.Tensor | None
    bjinv64: torch.Tensor | None
    bjinv32: torch.Tensor | None

    @property
    def nrows(self):
        return self.bsr.nrows

    @property
    def nnzb(self):
        return self.bsr.nnzb

    @property
    def nc(self):
        return self.bsr.nc

    @property
    def n(self):
        return self.bsr.nrows * self.bsr.nc

    def bytes(self):
        return sum(t.numel() * t.element_size() for t in
                   (self.row_ptr, self.col_idx, self.val64, self.val32, self.bjinv64, self.bjinv32)
                   if t is not None)


def assemble(spec, psi0: torch.Tensor | None, fp32: bool = True, block_jacobi: bool = True,
             device="cuda"):
    """dirac_st_assemble: returns (Operator, b).  psi0: complex128 [S*nc] on device."""
    nrows, nnzb = sizes(spec)
    nc = spec.nc
    dev = torch.device(device)
    rp = torch.empty(nrows + 1, dtype=torch.int32, device=dev)
    ci = torch.empty(nnzb, dtype=torch.int32, device=dev)
    v64 = torch.empty(nnzb * nc * nc, dtype=torch.complex128, device=dev)
    v32 = torch.empty(nnzb * nc * nc, dtype=torch.complex64, device=dev) if fp32 else None
    bj64 = torch.empty(nrows * nc * nc, dtype=torch.complex128, device=dev) if block_jacobi else None
    bj32 = torch.empty(nrows * nc * nc, dtype=torch.complex64, device=dev) if (block_jacobi and fp32) else None
    A = BSR()
    A.row_ptr, A.col_idx, A.val64 = rp.data_ptr(), ci.data_ptr(), v64.data_ptr()
    A.val32 = v32.data_ptr() if v32 is not None else None
    A.bjinv64 = bj64.data_ptr() if bj64 is not None else None
    A.bjinv32 = bj32.data_ptr() if bj32 is not None else None
    A.nrows, A.nnzb = nrows, nnzb
    b = None
    if psi0 is not None:
        assert psi0.dtype == torch.complex128 and psi0.is_contiguous() and psi0.numel() == spec.spatial * nc
        b = torch.empty(nrows * nc, dtype=torch.complex128, device=dev)
    p = make_problem(spec)
    _check(_lib.dirac_st_assemble(C.byref(p), _ptr(psi0), C.byref(A), _ptr(b), _stream()))
    return Operator(spec, A, rp, ci, v64, v32, bj64, bj32), b


def assemble_into(op: Operator, psi0: torch.Tensor | None, b: torch.Tensor | None) -> None:
    """dirac_st_assemble into the arrays of an existing Operator (same mesh)."""
    p = make_problem(op.spec)
    _check(_lib.dirac_st_assemble(C.byref(p), _ptr(psi0), C.byref(op.bsr), _ptr(b), _stream()))


def spmv(op: Operator, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    """dirac_st_spmv in the precision of x (complex128 -> 64, complex64 -> 32)."""
    prec = 64 if x.dtype == torch.complex128 else 32
    if y is None:
        y = torch.empty_like(x)
    _check(_lib.dirac_st_spmv(C.byref(op.bsr), prec, _ptr(x), _ptr(y), _stream()))
    return y


def spmv_mf(op_or_spec, x: torch.Tensor, y=None):
    """dirac_st_spmv_mf: y = A x from the problem alone (an Operator's problem,
    or a Spec)."""
    prob = op_or_spec.bsr.prob if isinstance(op_or_spec, Operator) else make_problem(op_or_spec)
    prec = 64 if x.dtype == torch.complex128 else 32
    if y is None:
        y = torch.empty_like(x)
    _check(_lib.dirac_st_spmv_mf(C.byref(prob), prec, _ptr(x), _ptr(y), _stream()))
    return y


def rhs_mf(spec, psi0: torch.Tensor, b=None):
    """dirac_st_rhs_mf: b = -D_w21 psi0 from the stencils (no assembly)."""
    prob = make_problem(spec)
    nrows, _ = sizes(spec)
    if b is None:
        b = torch.empty(nrows * spec.nc, dtype=torch.complex128, device=psi0.device)
    _check(_lib.dirac_st_rhs_mf(C.byref(prob), _ptr(psi0), _ptr(b), _stream()))
    return b


def slice_moments(spec, psi0: torch.Tensor, x: torch.Tensor, x_split: float) -> torch.Tensor:
    """dirac_st_slice_moments: [n_t + 1, 2 + d] float64 on the device (charge,
    charge past x_split, first moments per axis)."""
    prob = make_problem(spec)
    out = torch.empty((spec.n[0] + 1, 2 + spec.d), dtype=torch.float64, device=x.device)
    _check(_lib.dirac_st_slice_moments(C.byref(prob), _ptr(psi0), _ptr(x), float(x_split), _ptr(out), _stream()))
    return out


def problem_operator(spec) -> Operator:
    """An Operator with no stored arrays: only the problem, nc and the row count,
    for solves with matrix_free=True."""
    nrows, nnzb = sizes(spec)
    bsr = BSR()
    bsr.nrows, bsr.nnzb, bsr.nc = nrows, nnzb, spec.nc
    bsr.prob = make_problem(spec)
    return Operator(spec=spec, bsr=bsr, row_ptr=None, col_idx=None, val64=None, val32=None, bjinv64=None,
                    bjinv32=None)


def pc_apply(op: Operator, v: torch.Tensor, pc="spectral", vbar=0.0, z=None, work=None, slabs=1):
    prec = 64 if v.dtype == torch.complex128 else 32
    kind = PC_NAMES[pc] if isinstance(pc, str) else pc
    if z is None:
        z = torch.empty_like(v)
    o = Opts(restart=1, max_it=1, pc=kind, precision=prec, max_cycles=0, rtol=1e-8, inner_rtol=0.0,
             vbar=vbar, time_slabs=slabs)
    if kind in (PC_SPECTRAL, PC_LINE, PC_TIME_SLABS):
        nbytes = _lib.dirac_st_workspace_bytes(C.byref(op.bsr), C.byref(o), 0)
        if work is None or work.numel() < nbytes:
            work = torch.empty(nbytes, dtype=torch.uint8, device=v.device)
    _check(_lib.dirac_st_pc_apply(C.byref(op.bsr), C.byref(o), _ptr(v), _ptr(z), _ptr(work),
                                  work.numel() if work is not None else 0, _stream()))
    return z


def make_opts(restart=50, max_it=20000, pc="bj", precision=64, max_cycles=0, rtol=1e-8,
              inner_rtol=0.0, vbar=0.0, slabs=1, matrix_free=False) -> Opts:
    return Opts(restart=restart, max_it=max_it, pc=PC_NAMES[pc] if isinstance(pc, str) else pc,
                precision=precision, max_cycles=max_cycles, rtol=rtol, inner_rtol=inner_rtol,
                vbar=vbar, time_slabs=slabs, matrix_free=1 if matrix_free else 0)


def workspace_bytes(op: Operator, opts: Opts, flexible=False) -> int:
    return int(_lib.dirac_st_workspace_bytes(C.byref(op.bsr), C.byref(opts), 1 if flexible else 0))


def gmres(op: Operator, b: torch.Tensor, x: torch.Tensor | None = None, opts: Opts | None = None,
          work: torch.Tensor | None = None, history: int = 0, **kw):
    """dirac_st_gmres.  Returns (x, stats dict).  kw build the options when opts is None."""
    if opts is None:
        opts = make_opts(**kw)
    if x is None:
        x = torch.zeros_like(b)
    # room for the preconditioned vectors: one preconditioner application fewer per cycle
    nbytes = workspace_bytes(op, opts, flexible=True)
    if work is None or work.numel() < workspace_bytes(op, opts):
        work = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    st = Stats()
    hist = None
    if history:
        hist = (C.c_double * history)()
        st.history = C.cast(hist, C.POINTER(C.c_double))
        st.history_len = history
    rc = _lib.dirac_st_gmres(C.byref(op.bsr), _ptr(b), _ptr(x), C.byref(opts), _ptr(work),
                             work.numel(), C.byref(st), _stream())
    _check(rc, allow=(OK, NOT_CONVERGED))
    info = dict(rc=rc, iters=st.iters, cycles=st.cycles, converged=bool(st.converged),
                relres=st.relres, est=st.est, ms=st.ms, singular_blocks=st.singular_blocks)
    if hist is not None:
        info["history"] = [hist[i] for i in range(min(st.iters, history))]
    return x, info


def bicgstab(op: Operator, b: torch.Tensor, x: torch.Tensor | None = None, opts: Opts | None = None,
             work: torch.Tensor | None = None, history: int = 0, **kw):
    """dirac_st_bicgstab (complex128).  Returns (x, stats dict); kw build the
    options when opts is None (restart is ignored)."""
    if opts is None:
        opts = make_opts(**kw)
    if x is None:
        x = torch.zeros_like(b)
    if work is None:
        nbytes = int(_lib.dirac_st_bicgstab_workspace_bytes(C.byref(op.bsr), C.byref(opts)))
        work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=b.device)
    st = Stats()
    hist = None
    if history:
        hist = (C.c_double * history)()
        st.history = C.cast(hist, C.POINTER(C.c_double))
        st.history_len = history
    rc = _lib.dirac_st_bicgstab(C.byref(op.bsr), _ptr(b), _ptr(x), C.byref(opts), _ptr(work), work.numel(),
                                C.byref(st), _stream())
    _check(rc, allow=(OK, NOT_CONVERGED))
    info = dict(rc=rc, iters=st.iters, cycles=st.cycles, converged=bool(st.converged),
                relres=st.relres, est=st.est, ms=st.ms)
    if hist is not None:
        info["history"] = [hist[i] for i in range(min(st.iters, history))]
    return x, info


# ------------------------------------------------------------------ network
NN_PARAMS = int(_lib.dirac_st_nn_param_count())
NN_WEIGHTS = 27 * (4 * 16 + 16 * 16 + 16 * 16 + 16 * 4)


class Net:
    """Network parameters in device memory (FP32 master, bf16 copies, Adam state)."""

    def __init__(self, params, training=True):
        p = torch.as_tensor(params, dtype=torch.float32).reshape(-1).to("cuda").contiguous()
        assert p.numel() == NN_PARAMS
        self.params = p
        self.m = torch.zeros_like(p) if training else None
        self.v = torch.zeros_like(p) if training else None
        self.w16 = torch.empty(NN_WEIGHTS, dtype=torch.int16, device="cuda")
        self.wt16 = torch.empty(NN_WEIGHTS, dtype=torch.int16, device="cuda")
        self.s = NNStruct(params=p.data_ptr(), adam_m=self.m.data_ptr() if training else None,
                          adam_v=self.v.data_ptr() if training else None, w16=self.w16.data_ptr(),
                          wt16=self.wt16.data_ptr(), step=0, out_gain=1.0)
        _check(_lib.dirac_st_nn_pack(C.byref(self.s), _stream()))

    def repack(self):
        _check(_lib.dirac_st_nn_pack(C.byref(self.s), _stream()))


def nn_workspace_bytes(nt, ny, nx, training=False):
    return int(_lib.dirac_st_nn_workspace_bytes(nt, ny, nx, 1 if training else 0))


def _work(nbytes, work):
    if work is None or work.numel() < nbytes:
        work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
    return work


def nn_forward(net: Net, x: torch.Tensor, shape, scale=1.0, work=None):
    """x: float32 [nt*ny*nx*4] on device; shape (nt, ny, nx)."""
    nt, ny, nx = shape
    out = torch.empty_like(x)
    work = _work(nn_workspace_bytes(nt, ny, nx), work)
    _check(_lib.dirac_st_nn_forward(C.byref(net.s), nt, ny, nx, _ptr(x), scale, _ptr(out), _ptr(work),
                                    work.numel(), _stream()))
    return out


def nn_backward(net: Net, x, dout, shape, scale=1.0, work=None):
    nt, ny, nx = shape
    grad = torch.empty(NN_PARAMS, dtype=torch.float32, device="cuda")
    work = _work(nn_workspace_bytes(nt, ny, nx, True), work)
    _check(_lib.dirac_st_nn_backward(C.byref(net.s), nt, ny, nx, _ptr(x), scale, _ptr(dout), _ptr(grad),
                                     _ptr(work), work.numel(), _stream()))
    return grad


def nn_train_step(net: Net, x, target, shape, lr, loss_out=None, work=None):
    nt, ny, nx = shape
    work = _work(nn_workspace_bytes(nt, ny, nx, True), work)
    _check(_lib.dirac_st_nn_train_step(C.byref(net.s), nt, ny, nx, _ptr(x), _ptr(target), lr,
                                       _ptr(loss_out), _ptr(work), work.numel(), _stream()))
    return work


def fgmres_nn(op: Operator, b, net: Net | None, x=None, opts: Opts | None = None, work=None,
              history: int = 0, **kw):
    """dirac_st_fgmres_nn.  Returns (x, stats dict)."""
    if opts is None:
        opts = make_opts(**kw)
    if x is None:
        x = torch.zeros_like(b)
    nbytes = workspace_bytes(op, opts, flexible=True)
    work = _work(nbytes, work)
    st = Stats()
    hist = None
    if history:
        hist = (C.c_double * history)()
        st.history = C.cast(hist, C.POINTER(C.c_double))
        st.history_len = history
    rc = _lib.dirac_st_fgmres_nn(C.byref(op.bsr), _ptr(b), _ptr(x),
                                 C.byref(net.s) if net is not None else None, C.byref(opts),
                                 _ptr(work), work.numel(), C.byref(st), _stream())
    _check(rc, allow=(OK, NOT_CONVERGED))
    info = dict(rc=rc, iters=st.iters, cycles=st.cycles, converged=bool(st.converged),
                relres=st.relres, est=st.est, ms=st.ms, fallback=bool(st.fallback))
    if hist is not None:
        info["history"] = [hist[i] for i in range(min(st.iters, history))]
    return x, info


# ------------------------------------------------------------------ batches
def _bsr_array(ops):
    arr = (_BSRP * len(ops))()
    for i, op in enumerate(ops):
        arr[i] = C.pointer(op.bsr)
    return arr


def _ptr_array(ts):
    arr = (_vp * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


def batched_workspace_bytes(ops, opts: Opts) -> int:
    n = int(_lib.dirac_st_batched_workspace_bytes(len(ops), _bsr_array(ops), C.byref(opts)))
    if n == 0:
        raise DiracError(EINVAL, last_error())
    return n


def fgmres_batched(ops, bs, xs=None, opts: Opts | None = None, work=None, allow_breakdown=False, **kw):
    """dirac_st_fgmres_batched over the systems ops[i] x_i = b_i.  Returns (xs, list of stats
    dicts, rc).  Without opts, vbar defaults to -1 (each system uses half its step height).
    allow_breakdown: return EBREAKDOWN (some system hit NaN/Inf) instead of raising."""
    if opts is None:
        kw.setdefault("vbar", -1.0)
        opts = make_opts(**kw)
    if xs is None:
        xs = [torch.zeros_like(b) for b in bs]
    assert len(ops) == len(bs) == len(xs)
    A = _bsr_array(ops)
    nbytes = batched_workspace_bytes(ops, opts)
    work = _work(nbytes, work)
    st = (Stats * len(ops))()
    rc = _lib.dirac_st_fgmres_batched(len(ops), A, _ptr_array(bs), _ptr_array(xs), C.byref(opts),
                                      _ptr(work), work.numel(), st, _stream())
    _check(rc, allow=(OK, NOT_CONVERGED, EBREAKDOWN) if allow_breakdown else (OK, NOT_CONVERGED))
    infos = [dict(iters=s.iters, cycles=s.cycles, converged=bool(s.converged), relres=s.relres,
                  est=s.est, ms=s.ms) for s in st]
    return xs, infos, rc


def spmv_batched_workspace_bytes(ops) -> int:
    n = int(_lib.dirac_st_spmv_batched_workspace_bytes(len(ops), _bsr_array(ops)))
    if n == 0:
        raise DiracError(EINVAL, last_error())
    return n


def spmv_batched(ops, xs, ys=None, lanes=None, work=None):
    """dirac_st_spmv_batched: y_i = A_i x_i for every system in one launch."""
    prec = 64 if xs[0].dtype == torch.complex128 else 32
    if ys is None:
        ys = [torch.empty_like(x) for x in xs]
    if lanes is None:
        lanes = (32 if prec == 64 else 16) if ops[0].nc == 2 else 64
    A = _bsr_array(ops)
    nbytes = int(_lib.dirac_st_spmv_batched_workspace_bytes(len(ops), A))
    if nbytes == 0:
        raise DiracError(EINVAL, last_error())
    work = _work(nbytes, work)
    _check(_lib.dirac_st_spmv_batched(len(ops), A, prec, _ptr_array(xs), _ptr_array(ys),
                                      lanes, _ptr(work), work.numel(), _stream()))
    return ys


def batched_set_lanes(nc: int, prec: int, lanes: int) -> None:
    """Force the SpMV lanes per block row of the batched solver (0: autotune)."""
    _check(_lib.dirac_st_batched_set_lanes(nc, prec, lanes))


def batched_lanes(nc: int, prec: int, rows: int) -> int:
    """Lanes the batched solver uses for a batch of `rows` block rows (0: not tuned yet)."""
    return int(_lib.dirac_st_batched_lanes(nc, prec, rows))


def time_eigen(nt: int, ht: float):
    """dirac_st_time_eigen (host): (lam [nt], W [nt, nt], Q [nt, nt]) complex128 numpy arrays."""
    import numpy as np
    lam = np.zeros(nt, np.complex128)
    W = np.zeros((nt, nt), np.complex128)
    Q = np.zeros((nt, nt), np.complex128)
    _check(_lib.dirac_st_time_eigen(nt, ht, lam.ctypes.data, W.ctypes.data, Q.ctypes.data))
    return lam, W, Q


TIMED = {"spmv64": 0, "spmv32": 1, "resid64": 2, "assemble": 3}


def timing(on: bool) -> None:
    """dirac_st_timing: start (clearing earlier records) or stop kernel timing."""
    _check(_lib.dirac_st_timing(1 if on else 0))


def timing_read(kind: str):
    """dirac_st_timing_read: (launch count, total ms) of one timed kernel."""
    n, ms = _i64(0), C.c_double(0.0)
    _check(_lib.dirac_st_timing_read(TIMED[kind], C.byref(n), C.byref(ms)))
    return int(n.value), float(ms.value)
