"""ctypes wrapper of the plain FP64 CPU oracle (oracle/vlbm_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it to check and time the HIP library; nothing on the
product path imports it.  It shares no code with the HIP library.

The conventions the paper leaves open (see vlbm_oracle.h: a changing between
steps, the event counters, the outflow ghost layers, the sponge layer, wall
and Dirichlet ghosts and their corners) are pinned by
tests/test_oracle_conventions.py.

Layout conventions (float64 numpy arrays):
  state S   [20, ny, nx]  plane s*4 + c, slot s in (u, u_1, u_2, u_3, u_4),
                          component c in (rho, m1, m2, E)
  theta_x   [ny, nx + 1]  x-face between cells (i-1, j) and (i, j)
  theta_y   [ny + 1, nx]  y-face between cells (i, j-1) and (i, j)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SOURCES = [os.path.join(HERE, "vlbm_oracle.c")]
DEPS = SOURCES + [os.path.join(HERE, "model.inc"), os.path.join(HERE, "vlbm_oracle.h")]

BND_ZERO_GRADIENT, BND_WALL, BND_DIRICHLET = 0, 1, 2
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3
RHO_PP = 1
RHO_LMP = 2
RHO_RLMP = 4
PRESSURE = 8
A_DYNAMIC = 0
A_FIXED = 1
BLEND_FACE = 0
BLEND_CELL = 1
PERIODIC = 0
OUTFLOW = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2 -ffp-contract=off, no fast-math,
    OpenMP over rows (bit-identical to the serial loops)."""
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(p) for p in DEPS)
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unknown-pragmas",
           "-o", tmp] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("gamma", ctypes.c_double), ("alpha", ctypes.c_double),
        ("order", ctypes.c_int32), ("limiters", ctypes.c_uint32),
        ("a_mode", ctypes.c_int32),
        ("a_beta", ctypes.c_double), ("a_fixed", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("sponge", ctypes.c_int32),
        ("eps", ctypes.c_double), ("rlmp_lo", ctypes.c_double),
        ("rlmp_hi", ctypes.c_double),
        ("bnd_kind", ctypes.POINTER(ctypes.c_uint8) * 4),
        ("bnd_state", ctypes.POINTER(ctypes.c_double) * 4),
        ("blend", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("lam", ctypes.c_double), ("a", ctypes.c_double), ("dt", ctypes.c_double),
        ("kappa", ctypes.c_double), ("lambda_new", ctypes.c_double),
        ("n_guard", ctypes.c_int64), ("n_limited", ctypes.c_int64),
        ("n_bad", ctypes.c_int64), ("bouchut", ctypes.c_int32),
        ("n_lmp", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Params)
        ip = ctypes.POINTER(Info)
        L.orc_flux.argtypes = [dp, ctypes.c_double, dp, dp]
        L.orc_maxwellians.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_theta_rho_pp.argtypes = [ctypes.c_double] * 4
        L.orc_theta_rho_pp.restype = ctypes.c_double
        L.orc_theta_rho_lmp.argtypes = [ctypes.c_double] * 7
        L.orc_theta_rho_lmp.restype = ctypes.c_double
        L.orc_theta_p.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double]
        L.orc_theta_p.restype = ctypes.c_double
        L.orc_lambda.argtypes = [pp, dp, ctypes.POINTER(ctypes.c_int64)]
        L.orc_lambda.restype = ctypes.c_double
        L.orc_kinetic_speed.argtypes = [pp, ctypes.c_double]
        L.orc_kinetic_speed.restype = ctypes.c_double
        L.orc_init.argtypes = [pp, dp, dp, ip]
        L.orc_step.argtypes = [pp, dp, dp, dp, dp, ip]
        L.orc_run.argtypes = [pp, dp, dp, ctypes.c_int32, dp, ip, ctypes.POINTER(ctypes.c_int64)]
        L.orc_step_frozen.argtypes = [pp, dp, dp, dp, ctypes.c_double, dp]
        L.orc_step_frozen_cs.argtypes = [pp, dp, dp, dp, dp, ctypes.c_double, dp, dp]
        L.orc_init_frozen_cs.argtypes = [pp, dp, dp, ctypes.c_double, dp, dp]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Config:
    nx: int
    ny: int
    dx: float = None
    gamma: float = 1.4
    alpha: float = 0.5
    order: int = 2
    limiters: int = RHO_PP | PRESSURE
    a_mode: int = A_DYNAMIC
    a_beta: float = 1.0
    a_fixed: float = 0.0
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    sponge: int = 0
    eps: float = 1e-16
    rlmp_lo: float = 0.999
    rlmp_hi: float = 1.001
    # per-side (west, east, south, north) boundary kinds, uint8 [len] or None,
    # and Dirichlet moments, float64 [4, len] or None
    bnd_kind: tuple = (None, None, None, None)
    bnd_state: tuple = (None, None, None, None)
    # BLEND_FACE (Section 3.2) or BLEND_CELL (the per-cell blending of
    # Section 3.1, an ablation)
    blend: int = 0

    def params(self) -> Params:
        dx = self.dx if self.dx is not None else 1.0 / self.nx
        P = Params(self.nx, self.ny, dx, self.gamma, self.alpha, self.order,
                   self.limiters, self.a_mode, self.a_beta, self.a_fixed,
                   self.bc_x, self.bc_y, self.sponge, self.eps, self.rlmp_lo,
                   self.rlmp_hi)
        keep = []
        for side in range(4):
            k, st = self.bnd_kind[side], self.bnd_state[side]
            if k is not None:
                k = np.ascontiguousarray(k, dtype=np.uint8)
                keep.append(k)
                P.bnd_kind[side] = k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
            if st is not None:
                st = np.ascontiguousarray(st, dtype=np.float64)
                keep.append(st)
                P.bnd_state[side] = st.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        P.blend = self.blend
        P._keep = keep  # the arrays outlive the call that receives P
        return P


def flux(u, gamma=1.4):
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.zeros(4)
    g = np.zeros(4)
    lib().orc_flux(_p(u), gamma, _p(f), _p(g))
    return f, g


def maxwellians(u, a, gamma=1.4, alpha=0.5):
    """[5, 4]: M_1..M_5 of one state."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    M = np.zeros(20)
    lib().orc_maxwellians(_p(u), gamma, alpha, a, _p(M))
    return M.reshape(5, 4)


def theta_rho_pp(rho_star, D, kappa, eps=1e-16):
    return lib().orc_theta_rho_pp(rho_star, D, kappa, eps)


def theta_rho_lmp(rho_star, D, kappa, muL, nuL, muR, nuR):
    return lib().orc_theta_rho_lmp(rho_star, D, kappa, muL, nuL, muR, nuR)


def theta_p(ustar, dF, kappa, eps=1e-16):
    us = np.ascontiguousarray(ustar, dtype=np.float64)
    df = np.ascontiguousarray(dF, dtype=np.float64)
    return lib().orc_theta_p(_p(us), _p(df), kappa, eps)


def lam(cfg: Config, S):
    S = np.ascontiguousarray(S, dtype=np.float64)
    nbad = ctypes.c_int64(0)
    P = cfg.params()
    v = lib().orc_lambda(ctypes.byref(P), _p(S), ctypes.byref(nbad))
    return v, nbad.value


def kinetic_speed(cfg: Config, lam_):
    P = cfg.params()
    return lib().orc_kinetic_speed(ctypes.byref(P), lam_)


def init(cfg: Config, u0):
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    assert u0.shape == (4, cfg.ny, cfg.nx)
    S = np.empty((20, cfg.ny, cfg.nx))
    info = Info()
    P = cfg.params()
    rc = lib().orc_init(ctypes.byref(P), _p(u0), _p(S), ctypes.byref(info))
    if rc != 0:
        raise ValueError("oracle init failed (rc=%d, non-admissible cells %d)" % (rc, info.n_bad))
    return S, info


def step(cfg: Config, S):
    """One step; returns (S_new, theta_x, theta_y, info)."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    Sn = np.empty_like(S)
    tx = np.empty((cfg.ny, cfg.nx + 1))
    ty = np.empty((cfg.ny + 1, cfg.nx))
    info = Info()
    P = cfg.params()
    rc = lib().orc_step(ctypes.byref(P), _p(S), _p(Sn), _p(tx), _p(ty), ctypes.byref(info))
    if rc != 0:
        raise RuntimeError("oracle step failed (rc=%d)" % rc)
    return Sn, tx, ty, info


def run(cfg: Config, S, nsteps, t=0.0):
    """nsteps steps; returns (S_new, t_new, last_info, totals[guard, limited, bad, lmp])."""
    S = np.array(S, dtype=np.float64, order="C", copy=True)
    work = np.empty_like(S)
    tt = ctypes.c_double(t)
    info = Info()
    totals = (ctypes.c_int64 * 4)(0, 0, 0, 0)
    P = cfg.params()
    rc = lib().orc_run(ctypes.byref(P), _p(S), _p(work), int(nsteps), ctypes.byref(tt),
                       ctypes.byref(info), totals)
    if rc != 0:
        raise RuntimeError("oracle run failed (rc=%d)" % rc)
    return S, tt.value, info, tuple(totals)


def step_frozen(cfg: Config, S, theta_x, theta_y, a):
    S = np.ascontiguousarray(S, dtype=np.float64)
    Sn = np.empty_like(S)
    P = cfg.params()
    rc = lib().orc_step_frozen(ctypes.byref(P), _p(S), _p(np.ascontiguousarray(theta_x)),
                               _p(np.ascontiguousarray(theta_y)), a, _p(Sn))
    assert rc == 0
    return Sn


def step_frozen_cs(cfg: Config, S, Sim, theta_x, theta_y, a):
    S = np.ascontiguousarray(S, dtype=np.float64)
    Sim = np.ascontiguousarray(Sim, dtype=np.float64)
    Sn = np.empty_like(S)
    Sni = np.empty_like(S)
    P = cfg.params()
    rc = lib().orc_step_frozen_cs(ctypes.byref(P), _p(S), _p(Sim),
                                  _p(np.ascontiguousarray(theta_x)),
                                  _p(np.ascontiguousarray(theta_y)), a, _p(Sn), _p(Sni))
    assert rc == 0
    return Sn, Sni


def init_frozen_cs(cfg: Config, u0, u0_im, a):
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    u0_im = np.ascontiguousarray(u0_im, dtype=np.float64)
    S = np.empty((20, cfg.ny, cfg.nx))
    Sim = np.empty_like(S)
    P = cfg.params()
    rc = lib().orc_init_frozen_cs(ctypes.byref(P), _p(u0), _p(u0_im), a, _p(S), _p(Sim))
    assert rc == 0
    return S, Sim


def num_threads():
    return lib().orc_num_threads()
