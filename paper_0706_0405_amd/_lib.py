"""ctypes view of the C ABI declared in include/lbkt.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBKT_LIB") or os.path.join(HERE, "liblbkt.so")

LB_F64, LB_F32 = 0, 1
LB_ENONFINITE = -4
BC = {"periodic": 0, "outflow": 1, "wall": 2, "inflow": 3, "shock": 4}
FLAG_NONFINITE, FLAG_RHO_NONPOS, FLAG_T_NONPOS = 1, 2, 4


class LbState(ctypes.Structure):
    _fields_ = [("rho", c_double), ("ux", c_double), ("uy", c_double), ("p", c_double)]


class LbEdge(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("split", c_int32), ("a", LbState), ("b", LbState),
                ("x0", c_double), ("angle_deg", c_double), ("speed", c_double)]


class LbGrid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("pitch", c_int64), ("dx", c_double), ("dt", c_double),
                ("c1", c_double), ("c2", c_double), ("eta0", c_double), ("gamma", c_double),
                ("tau", c_double), ("beta", c_double), ("lam", c_double * 9), ("edge", LbEdge * 4)]


class LbTile(ctypes.Structure):
    _fields_ = [("block_x", c_int32), ("rows", c_int32), ("blocks", c_int32), ("steps", c_int32)]


class LbVnCase(ctypes.Structure):
    _fields_ = [("rho", c_double), ("ux", c_double), ("uy", c_double), ("T", c_double),
                ("c1", c_double), ("c2", c_double), ("eta0", c_double), ("gamma", c_double),
                ("tau", c_double), ("beta", c_double), ("dt", c_double), ("dx", c_double),
                ("lam", c_double * 9)]


class LbError(RuntimeError):
    def __init__(self, status, name, detail):
        super().__init__("%s (%d): %s" % (name, status, detail))
        self.status = status


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "lb_default_lambda": (c_int32, [POINTER(LbGrid)]),
    "lb_validate": (c_int32, [POINTER(LbGrid)]),
    "lb_array_elems": (c_int64, [POINTER(LbGrid)]),
    "lb_init": (c_int32, [POINTER(LbGrid), c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lb_step": (c_int32, [POINTER(LbGrid), c_int32, c_void_p, c_void_p, c_int64, c_void_p]),
    "lb_step_tiled": (c_int32, [POINTER(LbGrid), c_int32, c_void_p, c_void_p, c_int64, POINTER(LbTile), c_void_p]),
    "lb_run": (c_int32, [POINTER(LbGrid), c_int32, c_void_p, c_void_p, c_int64, c_int32, c_int32,
                         POINTER(LbTile), c_void_p]),
    "lb_moments": (c_int32, [POINTER(LbGrid), c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_void_p]),
    "lb_check_flags": (c_int32, [c_void_p, POINTER(c_uint32), c_void_p]),
    "lb_invariants": (c_int32, [POINTER(LbGrid), c_int32, c_void_p, c_void_p, c_void_p]),
    "lb_invariants_noalloc": (c_int32, [POINTER(LbGrid), c_int32, c_void_p, c_void_p, c_void_p]),
    "lb_step_adjoint": (c_int32, [POINTER(LbGrid), c_int32, c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
    "lb_run_record": (c_int32, [POINTER(LbGrid), c_int32, c_void_p, POINTER(c_void_p), c_int64, c_int32,
                                c_void_p]),
    "lb_adjoint_run": (c_int32, [POINTER(LbGrid), c_int32, POINTER(c_void_p), c_void_p, c_void_p, c_int64,
                                 c_int32, c_void_p]),
    "lb_init_adjoint": (c_int32, [POINTER(LbGrid), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p]),
    "lb_batch_create": (c_int32, [c_int32, POINTER(LbGrid), c_int32, POINTER(c_void_p)]),
    "lb_batch_layout": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)]),
    "lb_batch_set_tile": (c_int32, [c_void_p, POINTER(LbTile)]),
    "lb_step_batched": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "lb_batch_status": (c_int32, [c_void_p, c_void_p]),
    "lb_batch_destroy": (None, [c_void_p]),
    "lb_autotune": (c_int32, [POINTER(LbGrid), c_int32, c_void_p, c_void_p, c_int32, POINTER(LbTile),
                              POINTER(c_float), c_void_p]),
    "lb_vn_scan": (c_int32, [POINTER(LbVnCase), c_int32, c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "lb_vn_max_stable_dt": (c_int32, [POINTER(LbVnCase), c_int32, POINTER(c_double), c_int32, c_void_p, c_void_p,
                                      c_int32, c_double, POINTER(c_double), c_void_p]),
    "lb_struct_size": (c_int64, [c_int32]),
    "lb_status_str": (c_char_p, [c_int32]),
    "lb_last_error": (c_char_p, []),
}

EXPORTED = tuple(_SIGS)


def lib():
    """The loaded library; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbkt.so is not built (%s); run __graft_entry__.build() "
                               "or python -m paper_0706_0405_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        sizes = [L.lb_struct_size(i) for i in range(5)]
        want = [ctypes.sizeof(t) for t in (LbGrid, LbEdge, LbState, LbTile, LbVnCase)]
        if sizes != want:
            raise RuntimeError("ABI mismatch between lbkt.h and the ctypes structures: %s vs %s" % (sizes, want))
        _lib = L
    return _lib


def check(status):
    if status != 0:
        L = lib()
        raise LbError(status, L.lb_status_str(status).decode(), L.lb_last_error().decode())
    return status
