"""Owning wrappers around a library context: the workspace is a torch uint8
tensor on the current ROCm device and the context is bound to torch's current
stream.  Argument marshalling only; the method runs in libvlbm.so."""
from __future__ import annotations

import numpy as np

from . import binding as B


def _as_device(u, torch):
    if isinstance(u, np.ndarray):
        return torch.from_numpy(np.ascontiguousarray(u, dtype=np.float64)).cuda()
    return u.to(device="cuda", dtype=torch.float64).contiguous()


class Solver:
    """One instance.  Keyword arguments are the fields of lbm_params."""

    def __init__(self, u0, **kw):
        import torch

        u0 = _as_device(u0, torch)
        _, ny, nx = u0.shape
        self.params = B.make_params(nx, ny, **kw)
        nbytes = B.lbm_workspace_bytes(self.params)
        if nbytes == 0:
            raise ValueError("invalid parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.nx, self.ny = nx, ny
        self.ctx = B.lbm_init(self.params, u0, self.workspace)

    @property
    def dtype(self):
        import torch

        return torch.float64 if self.params.precision == B.LBM_FP64 else torch.float32

    def step(self, n=1):
        B.lbm_step(self.ctx, n)

    def step_graph(self, n):
        B.lbm_step_graph(self.ctx, n)

    def step_theta(self):
        """One step; returns (theta_x [ny, nx+1], theta_y [ny+1, nx])."""
        import torch

        tx = torch.empty((self.ny, self.nx + 1), dtype=torch.float64, device="cuda")
        ty = torch.empty((self.ny + 1, self.nx), dtype=torch.float64, device="cuda")
        B.lbm_step_theta(self.ctx, tx, ty)
        return tx, ty

    def moments(self, check=True):
        import torch

        out = torch.empty((4, self.ny, self.nx), dtype=torch.float64, device="cuda")
        st = B.lbm_moments(self.ctx, 0, out, check=check)
        return (out, st) if not check else out

    def diagnostics(self):
        return B.lbm_diagnostics(self.ctx, 0).as_dict()

    def totals(self):
        return B.lbm_totals(self.ctx, 0)

    def get_state(self):
        import torch

        s = torch.empty((20, self.ny, self.nx), dtype=self.dtype, device="cuda")
        B.lbm_get_state(self.ctx, s)
        return s

    def set_state(self, s):
        B.lbm_set_state(self.ctx, s.contiguous())

    def autotune(self, cache=None):
        """Pick (strip rows, waves per workgroup, groups per CU) by timing;
        returns the chosen launch."""
        B.lbm_autotune(self.ctx, cache)
        return self.launch()

    def set_launch(self, strip_rows=0, waves_per_group=0, groups_per_cu=None, strip_mode=None):
        B.lbm_set_launch(self.ctx, strip_rows, waves_per_group)
        if groups_per_cu is not None:
            B.lbm_set_grid(self.ctx, groups_per_cu)
        if strip_mode is not None:
            B.lbm_set_strip_mode(self.ctx, strip_mode)

    def launch(self):
        """(strip rows, waves per workgroup, groups per CU (0 = one wave per
        strip), strip mode (1 = heights matched to each instance))"""
        return B.lbm_get_launch(self.ctx) + (B.lbm_get_grid(self.ctx)[0], B.lbm_get_strip_mode(self.ctx))

    def set_boundary(self, side, kind=None, state=None):
        """Boundary cells of one side (B.LBM_WEST ... B.LBM_NORTH): kind uint8
        [len] (B.LBM_BND_*), state float64 [4, len] Dirichlet moments; numpy
        arrays are copied to the device and kept by the solver (update a
        moving state with set_boundary again, or in place on
        self.boundary[side][1])."""
        import torch

        if not hasattr(self, "boundary"):
            self.boundary = {}
        if kind is None:
            B.lbm_set_boundary(self.ctx, side)
            self.boundary.pop(side, None)
            return
        if isinstance(kind, np.ndarray):
            kind = torch.from_numpy(np.ascontiguousarray(kind, dtype=np.uint8)).cuda()
        k = kind.contiguous()  # the library keeps the pointer: hold this tensor
        st = None
        if state is not None:
            st = _as_device(state, torch).contiguous()
        B.lbm_set_boundary(self.ctx, side, k, st)
        self.boundary[side] = (k, st)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            B.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """Independent instances of uneven size advanced together (one launch per
    step).  u0s: list of [4, ny_i, nx_i] arrays; dx_i = 1/nx_i unless given."""

    def __init__(self, u0s, dx=None, **kw):
        import torch

        self.sizes = [(int(u.shape[2]), int(u.shape[1])) for u in u0s]
        nx = [s[0] for s in self.sizes]
        ny = [s[1] for s in self.sizes]
        packed = torch.cat([_as_device(u, torch).reshape(-1) for u in u0s])
        self.params = B.make_params(nx[0], ny[0], **kw)
        nbytes = B.lbm_batch_workspace_bytes(self.params, nx, ny)
        if nbytes == 0:
            raise ValueError("invalid parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.ctx = B.lbm_init_batch(self.params, nx, ny, packed, self.workspace, dx=dx)
        del packed

    def step(self, n=1):
        B.lbm_step(self.ctx, n)

    def step_graph(self, n):
        B.lbm_step_graph(self.ctx, n)

    def get_state(self):
        """Copy of the whole ensemble's state buffer (opaque bytes)."""
        import torch

        s = torch.empty(B.lbm_state_bytes(self.ctx), dtype=torch.uint8, device="cuda")
        B.lbm_get_state(self.ctx, s)
        return s

    def set_state(self, s):
        B.lbm_set_state(self.ctx, s.contiguous())

    def moments(self, inst, check=True):
        import torch

        nx, ny = self.sizes[inst]
        out = torch.empty((4, ny, nx), dtype=torch.float64, device="cuda")
        st = B.lbm_moments(self.ctx, inst, out, check=check)
        return (out, st) if not check else out

    def diagnostics(self, inst=0):
        return B.lbm_diagnostics(self.ctx, inst).as_dict()

    def totals(self, inst=0):
        return B.lbm_totals(self.ctx, inst)

    def autotune(self, cache=None):
        """Pick (strip rows, waves per workgroup, groups per CU) by timing;
        returns the chosen launch."""
        B.lbm_autotune(self.ctx, cache)
        return self.launch()

    def set_launch(self, strip_rows=0, waves_per_group=0, groups_per_cu=None, strip_mode=None):
        B.lbm_set_launch(self.ctx, strip_rows, waves_per_group)
        if groups_per_cu is not None:
            B.lbm_set_grid(self.ctx, groups_per_cu)
        if strip_mode is not None:
            B.lbm_set_strip_mode(self.ctx, strip_mode)

    def launch(self):
        """(strip rows, waves per workgroup, groups per CU (0 = one wave per
        strip), strip mode (1 = heights matched to each instance))"""
        return B.lbm_get_launch(self.ctx) + (B.lbm_get_grid(self.ctx)[0], B.lbm_get_strip_mode(self.ctx))

    def set_boundary(self, inst, side, kind=None, state=None):
        """Boundary cells of one side of instance `inst` (as Solver.set_boundary,
        sized by that instance); the device copies are kept in
        self.boundary[(inst, side)]."""
        import torch

        if not hasattr(self, "boundary"):
            self.boundary = {}
        if kind is None:
            B.lbm_set_instance_boundary(self.ctx, inst, side)
            self.boundary.pop((inst, side), None)
            return
        if isinstance(kind, np.ndarray):
            kind = torch.from_numpy(np.ascontiguousarray(kind, dtype=np.uint8)).cuda()
        k = kind.contiguous()
        st = None if state is None else _as_device(state, torch).contiguous()
        B.lbm_set_instance_boundary(self.ctx, inst, side, k, st)
        self.boundary[(inst, side)] = (k, st)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            B.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
