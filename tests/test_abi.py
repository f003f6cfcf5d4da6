"""The C ABI library loads on the host and exports every symbol that
include/vlbm.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

from paper_2411_15001_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "vlbm.h")).read()
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_exports_match_header():
    names = declared()
    assert set(names) == set(B.EXPORTS)
    L = ctypes.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_host_side_validation():
    L = B.lib()
    p = B.make_params(64, 64)
    assert B.lbm_workspace_bytes(p) > 20 * 64 * 64 * 8 * 2
    for bad in (dict(alpha=0.3), dict(gamma=1.0), dict(order=3), dict(a_beta=0.5),
                dict(limiters=16), dict(precision=2),
                dict(a_mode=1, a_fixed=0.0)):
        assert B.lbm_workspace_bytes(B.make_params(64, 64, **bad)) == 0, bad
    assert B.lbm_workspace_bytes(B.make_params(64, 64, alpha=0.3, unsafe=1)) > 0
    # FP32 state is half the size of FP64 state
    p32 = B.make_params(512, 512, precision=1)
    p64 = B.make_params(512, 512)
    assert B.lbm_workspace_bytes(p32) < B.lbm_workspace_bytes(p64)
    assert L.lbm_status_string(B.LBM_EPOSITIVITY) == b"non-admissible state"
    ctx = ctypes.c_void_p()
    st = L.lbm_init(ctypes.byref(p), None, None, None, ctypes.byref(ctx))
    assert st == B.LBM_EINVAL and not ctx.value
    assert B.lbm_last_error(None)
    assert L.lbm_step(None, 1) == B.LBM_EINVAL
    assert B.lbm_batch_workspace_bytes(p, [128, 256], [128, 256]) > 0
    assert B.lbm_batch_workspace_bytes(p, [128, 0], [128, 256]) == 0


def test_grid_size_limits():
    """Shapes the kernels cannot address are refused before any device work:
    sides of 2^30 or more and instances of 2^32 cells or more (32-bit cell
    offsets); the largest admissible shapes are accepted."""
    B.lib()
    ok = B.make_params(65536, 65535)  # 2^32 - 65536 cells
    assert B.lbm_workspace_bytes(ok) > 0
    assert B.lbm_workspace_bytes(B.make_params((1 << 30) - 1, 1)) > 0
    for nx, ny in ((65536, 65536), (70000, 70000), (1 << 30, 1), (1, 1 << 30), ((1 << 30) + 1, 1),
                   (0, 5), (5, 0)):
        assert B.lbm_workspace_bytes(B.make_params(nx, ny)) == 0, (nx, ny)
    p = B.make_params(128, 128)
    assert B.lbm_batch_workspace_bytes(p, [128, 256], [128, 256]) > 0
    assert B.lbm_batch_workspace_bytes(p, [128, 70000], [128, 70000]) == 0
    assert B.lbm_batch_workspace_bytes(p, [128, 64], [128, 0]) == 0
