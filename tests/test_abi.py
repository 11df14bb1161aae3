"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/lbkt.h declares, its structures match the binding, and host validation
rejects bad input before any launch. No GPU is needed."""
import ctypes
import os
import re

import pytest

from paper_0706_0405_amd import _lib
from paper_0706_0405_amd.api import Grid
from workloads import problems as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "lbkt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = _lib.lib()
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTED)


def test_struct_layout_matches_binding():
    L = _lib.lib()
    assert L.lb_struct_size(0) == ctypes.sizeof(_lib.LbGrid)
    assert L.lb_struct_size(1) == ctypes.sizeof(_lib.LbEdge)
    assert L.lb_struct_size(2) == ctypes.sizeof(_lib.LbState)
    assert L.lb_struct_size(3) == ctypes.sizeof(_lib.LbTile)
    assert L.lb_struct_size(4) == ctypes.sizeof(_lib.LbVnCase)
    assert L.lb_struct_size(9) == -1


def _grid(**kw):
    cfg = P.sod(nx=100, ny=4)
    cfg.update(kw)
    return Grid.from_workload(cfg)


def _status(g):
    return _lib.lib().lb_validate(ctypes.byref(g))


def test_default_lambda_is_eq13():
    g = _grid().c()
    lam = [g.lam[i] for i in range(9)]
    c1dx = g.c1 * g.dx
    assert lam == [c1dx] + [c1dx / 10.0] * 4 + [0.0] * 4


def test_validate_accepts_workloads():
    for cfg in (P.sod(), P.ratio1000(), P.regular_reflection(), P.double_mach(), P.roofline_grid(),
                P.periodic_smooth()):
        assert _status(Grid.from_workload(cfg).c()) == 0


@pytest.mark.parametrize("field,value,status", [
    ("c2", 1.0, -2),           # c1 == c2 is singular in Eqs. (e17)-(e18)
    ("beta", 0.6, -2),
    ("beta", -0.1, -2),
    ("tau", 0.0, -2),
    ("gamma", 1.0, -2),
    ("dt", -1.0, -2),
    ("eta0", 0.0, -2),
])
def test_validate_rejects_parameters(field, value, status):
    cfg = P.sod(nx=100, ny=4)
    cfg[field] = value
    assert _status(Grid.from_workload(cfg).c()) == status


def test_validate_rejects_layout_and_edges():
    g = _grid().c()
    g.pitch = 100                                 # not a multiple of 64
    assert _status(g) == -1
    g = _grid().c()
    g.nx = 0
    assert _status(g) == -1
    g = _grid().c()
    g.edge[0].kind = _lib.BC["periodic"]          # only one periodic x edge
    assert _status(g) == -2
    g = _grid().c()
    g.edge[0].kind = _lib.BC["shock"]             # shock edges are y edges
    assert _status(g) == -2
    g = _grid().c()
    g.lam[2] = 0.5                                # lambda differs inside the axis group
    assert _status(g) == -7
    g = _grid().c()
    g.edge[2].split = 3                           # split on a periodic edge
    assert _status(g) == -2
    cfg = P.double_mach(nx=96, ny=24)
    g = Grid.from_workload(cfg).c()
    g.edge[3].b.rho = -1.0                        # bad shock state
    assert _status(g) == -2
    g = _grid(nx=(1 << 27) + 1, ny=1).c()         # pitch beyond 2^27 elements
    assert _status(g) == -7
    g = _grid(nx=8192 * 8, ny=2048).c()           # 9 planes over 4 GiB: accepted
    assert _status(g) == 0


def test_batched_problem_over_4_gib_rejected():
    L = _lib.lib()
    grids = (_lib.LbGrid * 2)(_grid().c(), _grid(nx=8192 * 8, ny=2048).c())
    out = ctypes.c_void_p()
    assert L.lb_batch_create(2, grids, 0, ctypes.byref(out)) == -7
    assert b"4 GiB" in L.lb_last_error() and not out.value


def test_tile_steps_validated_before_launch():
    """lb_tile.steps (time steps per pass of lb_run) must be 0, 1, 2 or 3, and 3 runs
    on FP64 arrays with at least 3 rows only (LB_EUNSUPPORTED otherwise)."""
    L = _lib.lib()
    g = _grid().c()
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)   # never dereferenced
    for steps, want in ((4, -1), (-1, -1)):
        t = _lib.LbTile(0, 0, 0, steps)
        st = L.lb_run(ctypes.byref(g), 0, a, b, 0, 4, 0, ctypes.byref(t), None)
        assert st == want and b"steps" in L.lb_last_error()
    t = _lib.LbTile(0, 0, 0, 3)
    assert L.lb_run(ctypes.byref(g), 1, a, b, 0, 4, 0, ctypes.byref(t), None) == -7   # FP32 storage
    assert b"three steps" in L.lb_last_error()
    g2 = _grid(ny=2).c()
    assert L.lb_run(ctypes.byref(g2), 0, a, b, 0, 4, 0, ctypes.byref(t), None) == -7   # two rows
    assert b"three steps" in L.lb_last_error()


def test_alias_and_alignment_rejected_before_launch():
    L = _lib.lib()
    g = _grid().c()
    buf = ctypes.c_void_p(1 << 20)   # never dereferenced: the call returns before any launch
    st = L.lb_step(ctypes.byref(g), 0, buf, buf, 0, None)
    assert st == -3 and b"overlap" in L.lb_last_error()
    st = L.lb_step(ctypes.byref(g), 0, ctypes.c_void_p((1 << 20) + 8), ctypes.c_void_p(1 << 30), 0, None)
    assert st == -1 and b"aligned" in L.lb_last_error()
    st = L.lb_step(ctypes.byref(g), 7, buf, ctypes.c_void_p(1 << 30), 0, None)
    assert st == -1
    assert L.lb_status_str(-4) == b"LB_ENONFINITE"
    assert L.lb_check_flags(None, None, None) == -1 and b"NULL" in L.lb_last_error()


def test_run_record_arguments_rejected_before_launch():
    """lb_run_record checks every output (alignment, overlap of consecutive states)
    before its first launch."""
    L = _lib.lib()
    g = _grid().c()
    f0 = ctypes.c_void_p(1 << 20)   # never dereferenced
    A, B, C = 1 << 30, 1 << 31, 1 << 32

    def outs(*ptrs):
        return (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(p) for p in ptrs])

    assert L.lb_run_record(ctypes.byref(g), 0, f0, outs(A), 0, -1, None) == -1
    assert L.lb_run_record(ctypes.byref(g), 0, f0, None, 0, 2, None) == -1
    st = L.lb_run_record(ctypes.byref(g), 0, f0, outs(A, B + 8, C), 0, 3, None)
    assert st == -1 and b"aligned" in L.lb_last_error()
    st = L.lb_run_record(ctypes.byref(g), 0, f0, outs(A, B, B), 0, 3, None)
    assert st == -3 and b"overlap" in L.lb_last_error()
    st = L.lb_run_record(ctypes.byref(g), 0, f0, outs(1 << 20, A), 0, 2, None)
    assert st == -3 and b"overlap" in L.lb_last_error()


def test_array_elems():
    g = _grid(nx=100, ny=4).c()
    assert g.pitch == 128
    assert _lib.lib().lb_array_elems(ctypes.byref(g)) == 9 * 128 * 4


def _vn_case(**kw):
    from paper_0706_0405_amd import vn
    c = vn.case(_grid(), (1.0, 0.1, 0.0, 0.5))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_vn_scan_rejects_bad_arguments_before_launch():
    """Every check of lb_vn_scan / lb_vn_max_stable_dt happens on the host, before
    any device call (the k pointers are never dereferenced here)."""
    L = _lib.lib()
    k = ctypes.c_void_p(1 << 20)
    out = ctypes.c_void_p(1 << 21)
    one = (_lib.LbVnCase * 1)(_vn_case())
    assert L.lb_vn_scan(one, 0, k, k, 4, 0, out, None) == -1
    assert L.lb_vn_scan(one, 1, k, k, 0, 0, out, None) == -1
    assert L.lb_vn_scan(one, 1, None, k, 4, 0, out, None) == -1
    assert L.lb_vn_scan(one, 1, k, k, 4, 0, None, None) == -1
    assert L.lb_vn_scan(one, 1 << 16, k, k, 1 << 16, 0, out, None) == -1      # 2^32 points
    for bad in (dict(rho=0.0), dict(T=-1.0), dict(ux=float("nan")), dict(c2=1.0), dict(c1=1.0, c2=1.0),
                dict(beta=0.7), dict(tau=0.0), dict(gamma=1.0), dict(dt=-1.0)):
        two = (_lib.LbVnCase * 2)(_vn_case(), _vn_case(**bad))
        if "c2" in bad and "c1" not in bad:
            two[1].c1 = 1.0
        st = L.lb_vn_scan(two, 2, k, k, 4, 0, out, None)
        assert st == -2, bad
        assert b"case 1" in L.lb_last_error(), bad
    dts = (ctypes.c_double * 3)(0.1, 0.05, 0.2)                                  # not ascending
    res = (ctypes.c_double * 2)()
    assert L.lb_vn_max_stable_dt(one, 1, dts, 3, k, k, 4, 1e-12, res, None) == -1
    two = (_lib.LbVnCase * 2)(_vn_case(), _vn_case())
    dts = (ctypes.c_double * 4)(0.01, 0.02, 0.03, 0.03)                          # case 1 not ascending
    assert L.lb_vn_max_stable_dt(two, 2, dts, 2, k, k, 4, 1e-12, res, None) == -1
    assert b"case 1" in L.lb_last_error()
    dts = (ctypes.c_double * 2)(0.01, 0.02)
    assert L.lb_vn_max_stable_dt(one, 1, dts, 2, k, k, 4, -1.0, res, None) == -1
    assert L.lb_vn_max_stable_dt(one, 1, dts, 0, k, k, 4, 0.0, res, None) == -1
    assert L.lb_vn_max_stable_dt(one, 1, None, 2, k, k, 4, 0.0, res, None) == -1
