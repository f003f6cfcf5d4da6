"""ctypes binding of libvlbm.so (include/vlbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  Device memory comes from torch tensors on a ROCm device and
the stream is torch's current stream.  If the library has not been built the
import of a binding function raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvlbm.so")

LBM_OK = 0
LBM_EINVAL = 1
LBM_ENOTSUP = 2
LBM_EDEVICE = 3
LBM_EPOSITIVITY = 4
LBM_ENONFINITE = 5
LBM_EBOUCHUT = 6
LBM_EGUARD = 7

LBM_RHO_PP = 1
LBM_RHO_LMP = 2
LBM_RHO_RLMP = 4
LBM_PRESSURE = 8
LBM_A_DYNAMIC = 0
LBM_A_FIXED = 1
LBM_BC_PERIODIC = 0
LBM_BC_OUTFLOW = 1
LBM_BND_ZERO_GRADIENT = 0
LBM_BND_WALL = 1
LBM_BND_DIRICHLET = 2
LBM_WEST, LBM_EAST, LBM_SOUTH, LBM_NORTH = 0, 1, 2, 3
LBM_FP64 = 0
LBM_FP32_STATE = 1
LBM_BLEND_FACE = 0
LBM_BLEND_CELL = 1

EXPORTS = [
    "lbm_workspace_bytes", "lbm_batch_workspace_bytes", "lbm_init", "lbm_init_batch",
    "lbm_step", "lbm_step_graph", "lbm_step_theta", "lbm_moments", "lbm_diagnostics",
    "lbm_totals",
    "lbm_state_bytes", "lbm_get_state", "lbm_set_state", "lbm_step_between", "lbm_step_adjoint",
    "lbm_step_adjoint_theta", "lbm_init_adjoint", "lbm_autotune", "lbm_set_launch", "lbm_get_launch",
    "lbm_set_grid", "lbm_get_grid", "lbm_set_strip_mode", "lbm_get_strip_mode", "lbm_set_boundary",
    "lbm_set_instance_boundary", "lbm_step_noalloc",
    "lbm_status_string", "lbm_last_error", "lbm_destroy",
]


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double), ("gamma", ctypes.c_double), ("alpha", ctypes.c_double),
        ("order", ctypes.c_int32), ("limiters", ctypes.c_uint32),
        ("a_mode", ctypes.c_int32),
        ("a_beta", ctypes.c_double), ("a_fixed", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("sponge", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("eps", ctypes.c_double), ("rlmp_lo", ctypes.c_double), ("rlmp_hi", ctypes.c_double),
        ("unsafe", ctypes.c_int32),
        ("blend", ctypes.c_int32),
    ]


class lbm_diag(ctypes.Structure):
    _fields_ = [
        ("lam", ctypes.c_double), ("a", ctypes.c_double), ("t", ctypes.c_double),
        ("step", ctypes.c_int64), ("n_guard", ctypes.c_int64),
        ("n_limited", ctypes.c_int64), ("n_bad", ctypes.c_int64),
        ("bouchut", ctypes.c_int32), ("n_lmp", ctypes.c_int64),
        ("n_nonfinite", ctypes.c_int64), ("n_rho", ctypes.c_int64), ("n_rhoe", ctypes.c_int64),
        ("min_rho", ctypes.c_double), ("min_rhoe", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvlbm.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2411_15001_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        pp = ctypes.POINTER(lbm_params)
        i32 = ctypes.c_int32
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.lbm_workspace_bytes.argtypes = [pp]
        L.lbm_workspace_bytes.restype = ctypes.c_size_t
        L.lbm_batch_workspace_bytes.argtypes = [pp, i32, i32p, i32p]
        L.lbm_batch_workspace_bytes.restype = ctypes.c_size_t
        L.lbm_init.argtypes = [pp, vp, vp, vp, ctypes.POINTER(vp)]
        L.lbm_init_batch.argtypes = [pp, i32, i32p, i32p, ctypes.POINTER(ctypes.c_double), vp, vp,
                                     vp, ctypes.POINTER(vp)]
        L.lbm_step.argtypes = [vp, i32]
        L.lbm_step_graph.argtypes = [vp, i32]
        L.lbm_step_theta.argtypes = [vp, vp, vp]
        L.lbm_moments.argtypes = [vp, i32, vp]
        L.lbm_diagnostics.argtypes = [vp, i32, ctypes.POINTER(lbm_diag)]
        L.lbm_totals.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
        L.lbm_state_bytes.argtypes = [vp]
        L.lbm_state_bytes.restype = ctypes.c_size_t
        L.lbm_get_state.argtypes = [vp, vp]
        L.lbm_set_state.argtypes = [vp, vp]
        L.lbm_step_adjoint.argtypes = [vp, vp, vp, vp]
        L.lbm_step_adjoint_theta.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lbm_step_between.argtypes = [vp, vp, vp, vp, vp]
        L.lbm_init_adjoint.argtypes = [vp, vp, vp, vp]
        L.lbm_autotune.argtypes = [vp, ctypes.c_char_p]
        L.lbm_set_launch.argtypes = [vp, i32, i32]
        L.lbm_get_launch.argtypes = [vp, i32p, i32p]
        L.lbm_set_grid.argtypes = [vp, i32]
        L.lbm_set_strip_mode.argtypes = [vp, i32]
        L.lbm_set_boundary.argtypes = [vp, i32, vp, vp]
        L.lbm_set_instance_boundary.argtypes = [vp, i32, i32, vp, vp]
        L.lbm_get_strip_mode.argtypes = [vp, i32p]
        L.lbm_step_noalloc.argtypes = [pp, vp, vp, vp, ctypes.POINTER(lbm_diag)]
        L.lbm_get_grid.argtypes = [vp, i32p, i32p]
        L.lbm_status_string.argtypes = [ctypes.c_int]
        L.lbm_status_string.restype = ctypes.c_char_p
        L.lbm_last_error.argtypes = [vp]
        L.lbm_last_error.restype = ctypes.c_char_p
        L.lbm_destroy.argtypes = [vp]
        L.lbm_destroy.restype = None
        for name in EXPORTS:
            f = getattr(L, name)
            if f.restype is ctypes.c_int:  # the default: status codes
                f.restype = ctypes.c_int
        _lib = L
    return _lib


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (%d): %s" % (lib().lbm_status_string(status).decode(), status, message))
        self.status = status


def _check(status, ctx=None):
    if status != LBM_OK:
        msg = lib().lbm_last_error(ctx).decode()
        raise LbmError(status, msg)
    return status


def make_params(nx, ny, dx=None, gamma=1.4, alpha=0.5, order=2,
                limiters=LBM_RHO_PP | LBM_PRESSURE, a_mode=LBM_A_DYNAMIC, a_beta=1.0,
                a_fixed=0.0, bc_x=LBM_BC_PERIODIC, bc_y=LBM_BC_PERIODIC, sponge=0,
                precision=LBM_FP64, eps=1e-16, rlmp_lo=0.999, rlmp_hi=1.001,
                unsafe=0, blend=0):
    if dx is None:
        dx = 1.0 / nx if nx > 0 else 1.0  # nx < 1 is refused by the library
    return lbm_params(nx, ny, dx, gamma, alpha, order, limiters,
                      a_mode, a_beta, a_fixed, bc_x, bc_y, sponge, precision, eps, rlmp_lo,
                      rlmp_hi, unsafe, blend)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_cuda(t, dtype=None, numel=None, name="tensor"):
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise ValueError("%s: expected a contiguous device tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s: expected dtype %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s: expected %d elements, got %d" % (name, numel, t.numel()))


# (nx, ny) of every instance of each live context, keyed by the handle value;
# the bindings check tensor sizes against it before a pointer reaches the
# library (the C entry points take bare pointers).
_shapes = {}


def _inst_shape(ctx, inst=0):
    sh = _shapes.get(ctx.value if isinstance(ctx, ctypes.c_void_p) else ctx)
    if sh is None:
        raise ValueError("unknown or destroyed context")
    if not 0 <= inst < len(sh):
        raise ValueError("instance index out of range")
    return sh[inst]


# --------------------------------------------------------------------------
# Functions with the names of the C ABI
# --------------------------------------------------------------------------

def lbm_workspace_bytes(params):
    return lib().lbm_workspace_bytes(ctypes.byref(params))


def lbm_batch_workspace_bytes(params, nx, ny):
    n = len(nx)
    ax = (ctypes.c_int32 * n)(*nx)
    ay = (ctypes.c_int32 * n)(*ny)
    return lib().lbm_batch_workspace_bytes(ctypes.byref(params), n, ax, ay)


def lbm_init(params, u0, workspace):
    import torch

    _require_cuda(u0, torch.float64, 4 * params.nx * params.ny, "u0")
    _require_cuda(workspace)
    need = lbm_workspace_bytes(params)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError("workspace: %d bytes needed" % need)
    ctx = ctypes.c_void_p()
    _check(lib().lbm_init(ctypes.byref(params), _ptr(u0), _ptr(workspace), _stream(),
                          ctypes.byref(ctx)))
    _shapes[ctx.value] = [(params.nx, params.ny)]
    return ctx


def lbm_init_batch(params, nx, ny, u0_packed, workspace, dx=None):
    import torch

    _require_cuda(u0_packed, torch.float64, 4 * sum(a * b for a, b in zip(nx, ny)), "u0_packed")
    _require_cuda(workspace)
    need = lbm_batch_workspace_bytes(params, nx, ny)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError("workspace: %d bytes needed" % need)
    n = len(nx)
    ax = (ctypes.c_int32 * n)(*nx)
    ay = (ctypes.c_int32 * n)(*ny)
    adx = (ctypes.c_double * n)(*dx) if dx is not None else None
    ctx = ctypes.c_void_p()
    _check(lib().lbm_init_batch(ctypes.byref(params), n, ax, ay, adx, _ptr(u0_packed),
                                _ptr(workspace), _stream(), ctypes.byref(ctx)))
    _shapes[ctx.value] = [(int(a), int(b)) for a, b in zip(nx, ny)]
    return ctx


def lbm_step(ctx, nsteps):
    return _check(lib().lbm_step(ctx, int(nsteps)), ctx)


def lbm_step_graph(ctx, nsteps):
    return _check(lib().lbm_step_graph(ctx, int(nsteps)), ctx)


def lbm_step_theta(ctx, theta_x, theta_y):
    import torch

    nx, ny = _inst_shape(ctx)
    _require_cuda(theta_x, torch.float64, ny * (nx + 1), "theta_x")
    _require_cuda(theta_y, torch.float64, (ny + 1) * nx, "theta_y")
    return _check(lib().lbm_step_theta(ctx, _ptr(theta_x), _ptr(theta_y)), ctx)


def lbm_step_between(ctx, src, dst, theta_x=None, theta_y=None):
    """One step from the state in src to dst (caller buffers); see the C
    declaration for the context's state afterwards."""
    import torch

    _require_cuda(src)
    _require_state_bytes(ctx, src)
    _require_cuda(dst)
    _require_state_bytes(ctx, dst)
    if (theta_x is None) != (theta_y is None):
        raise ValueError("give both theta buffers or neither")
    tx = ty = None
    if theta_x is not None:
        nx, ny = _inst_shape(ctx)
        _require_cuda(theta_x, torch.float64, ny * (nx + 1), "theta_x")
        _require_cuda(theta_y, torch.float64, (ny + 1) * nx, "theta_y")
        tx, ty = _ptr(theta_x), _ptr(theta_y)
    return _check(lib().lbm_step_between(ctx, _ptr(src), _ptr(dst), tx, ty), ctx)


def lbm_step_noalloc(params, src, dst, diag=True, check=True):
    """One step of a single instance from the state in src to dst (device
    tensors of 20 * nx * ny elements of the params' precision) without a
    context; returns (status, lbm_diag or None).  With diag=False the call is
    asynchronous on torch's current stream."""
    import torch

    dt = torch.float64 if params.precision == LBM_FP64 else torch.float32
    n = 20 * params.nx * params.ny
    _require_cuda(src, dt, n, "src")
    _require_cuda(dst, dt, n, "dst")
    d = lbm_diag() if diag else None
    st = lib().lbm_step_noalloc(ctypes.byref(params), _ptr(src), _ptr(dst), _stream(),
                                ctypes.byref(d) if diag else None)
    if check:
        _check(st, None)
    return st, d


def lbm_moments(ctx, inst, out, check=True):
    import torch

    nx, ny = _inst_shape(ctx, int(inst))
    _require_cuda(out, torch.float64, 4 * nx * ny, "out")
    st = lib().lbm_moments(ctx, int(inst), _ptr(out))
    if check:
        _check(st, ctx)
    return st


def lbm_diagnostics(ctx, inst=0):
    d = lbm_diag()
    _check(lib().lbm_diagnostics(ctx, int(inst), ctypes.byref(d)), ctx)
    return d


def lbm_totals(ctx, inst=0):
    """(sum rho, sum m1, sum m2, sum E) of instance inst, compensated sums."""
    _inst_shape(ctx, int(inst))
    out = (ctypes.c_double * 4)()
    _check(lib().lbm_totals(ctx, int(inst), out), ctx)
    return tuple(out)


def lbm_state_bytes(ctx):
    return lib().lbm_state_bytes(ctx)


def _require_state_bytes(ctx, t):
    need = lbm_state_bytes(ctx)
    have = t.numel() * t.element_size()
    if not t.is_contiguous() or have != need:
        raise ValueError("state tensor must be contiguous and hold exactly %d bytes (got %d)"
                         % (need, have))


def lbm_get_state(ctx, dst):
    _require_cuda(dst)
    _require_state_bytes(ctx, dst)
    return _check(lib().lbm_get_state(ctx, _ptr(dst)), ctx)


def lbm_set_state(ctx, src):
    _require_cuda(src)
    _require_state_bytes(ctx, src)
    return _check(lib().lbm_set_state(ctx, _ptr(src)), ctx)


def lbm_step_adjoint(ctx, U_n, Ubar_np1, Ubar_n):
    import torch

    nx, ny = _inst_shape(ctx)
    for t, name in ((U_n, "U_n"), (Ubar_np1, "Ubar_np1"), (Ubar_n, "Ubar_n")):
        _require_cuda(t, torch.float64, 20 * nx * ny, name)
    return _check(lib().lbm_step_adjoint(ctx, _ptr(U_n), _ptr(Ubar_np1), _ptr(Ubar_n)), ctx)


def lbm_step_adjoint_theta(ctx, U_n, theta_x, theta_y, Ubar_np1, Ubar_n):
    import torch

    nx, ny = _inst_shape(ctx)
    for t, name in ((U_n, "U_n"), (Ubar_np1, "Ubar_np1"), (Ubar_n, "Ubar_n")):
        _require_cuda(t, torch.float64, 20 * nx * ny, name)
    _require_cuda(theta_x, torch.float64, ny * (nx + 1), "theta_x")
    _require_cuda(theta_y, torch.float64, (ny + 1) * nx, "theta_y")
    return _check(lib().lbm_step_adjoint_theta(ctx, _ptr(U_n), _ptr(theta_x), _ptr(theta_y),
                                               _ptr(Ubar_np1), _ptr(Ubar_n)), ctx)


def lbm_init_adjoint(ctx, u0, Ubar0, u0bar):
    import torch

    nx, ny = _inst_shape(ctx)
    for t, name, k in ((u0, "u0", 4), (Ubar0, "Ubar0", 20), (u0bar, "u0bar", 4)):
        _require_cuda(t, torch.float64, k * nx * ny, name)
    return _check(lib().lbm_init_adjoint(ctx, _ptr(u0), _ptr(Ubar0), _ptr(u0bar)), ctx)


def lbm_autotune(ctx, cache_path=None):
    p = cache_path.encode() if cache_path else None
    return _check(lib().lbm_autotune(ctx, p), ctx)


def lbm_set_launch(ctx, strip_rows=0, waves_per_group=0):
    return _check(lib().lbm_set_launch(ctx, int(strip_rows), int(waves_per_group)), ctx)


def lbm_get_launch(ctx):
    r = ctypes.c_int32()
    w = ctypes.c_int32()
    _check(lib().lbm_get_launch(ctx, ctypes.byref(r), ctypes.byref(w)), ctx)
    return r.value, w.value


def lbm_set_grid(ctx, groups_per_cu=0):
    return _check(lib().lbm_set_grid(ctx, int(groups_per_cu)), ctx)


def lbm_set_strip_mode(ctx, mode=0):
    return _check(lib().lbm_set_strip_mode(ctx, int(mode)), ctx)


def _boundary_ptrs(ctx, inst, side, kind, state):
    import torch

    sh = _shapes.get(ctx.value if isinstance(ctx, ctypes.c_void_p) else ctx)
    if sh is None:
        raise ValueError("unknown or destroyed context")
    # an instance index out of range goes to the library unchecked, which
    # rejects it (LBM_EINVAL) before reading any description
    n = None
    if 0 <= int(inst) < len(sh):
        nx, ny = sh[int(inst)]
        n = ny if int(side) in (0, 1) else nx
    kp = sp = None
    if kind is not None:
        _require_cuda(kind, torch.uint8, n, "kind")
        kp = _ptr(kind)
        if state is not None:
            _require_cuda(state, torch.float64, None if n is None else 4 * n, "state")
            sp = _ptr(state)
    return kp, sp


def lbm_set_boundary(ctx, side, kind=None, state=None):
    """Boundary cells of one side (0 west, 1 east, 2 south, 3 north): kind a
    uint8 device tensor of the side's length (LBM_BND_*), state float64
    [4, len] device tensor of Dirichlet moments (or None); kind None restores
    zero-gradient cells.  The tensors must outlive the context's steps."""
    kp, sp = _boundary_ptrs(ctx, 0, side, kind, state)
    return _check(lib().lbm_set_boundary(ctx, int(side), kp, sp), ctx)


def lbm_set_instance_boundary(ctx, inst, side, kind=None, state=None):
    """lbm_set_boundary for instance `inst` of an ensemble."""
    kp, sp = _boundary_ptrs(ctx, inst, side, kind, state)
    return _check(lib().lbm_set_instance_boundary(ctx, int(inst), int(side), kp, sp), ctx)


def lbm_get_strip_mode(ctx):
    m = ctypes.c_int32()
    _check(lib().lbm_get_strip_mode(ctx, ctypes.byref(m)), ctx)
    return m.value


def lbm_get_grid(ctx):
    """(groups per compute unit, 0 = one wave per strip; workgroups per launch)"""
    k = ctypes.c_int32()
    g = ctypes.c_int32()
    _check(lib().lbm_get_grid(ctx, ctypes.byref(k), ctypes.byref(g)), ctx)
    return k.value, g.value


def lbm_last_error(ctx=None):
    return lib().lbm_last_error(ctx).decode()


def lbm_destroy(ctx):
    _shapes.pop(ctx.value if isinstance(ctx, ctypes.c_void_p) else ctx, None)
    lib().lbm_destroy(ctx)
