"""ctypes wrapper of the CPU oracle (oracle.c).

TEST INFRASTRUCTURE: imported only by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The device library never imports, links or
calls anything here, and this package never touches the device library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OPS_ALL = 0x1F
OPS_EXT = 0xE0  # segment relocate (op 5), reversed relocate (op 6), cross-exchange (ops 7..9)
NOT_A_MOVE = 0xFF


def id_span(op_mask: int) -> int:
    """Move ids are below id_span * Q^2: 20 for operators 0..4, 40 with the
    operator variants (ops 5..9)."""
    return 40 if op_mask & OPS_EXT else 20


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-pthread", "-shared", "-fPIC",
                               "-Wall", "-Wno-unused-function", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        lib.oracle_eval.restype = ctypes.c_int
        lib.oracle_eval.argtypes = [i32, P, P, i64, i32, i32, P, P, u32, i32, P, P, P, P, P]
        lib.oracle_apply.restype = ctypes.c_int
        lib.oracle_apply.argtypes = [i32, P, P, i64, i32, i32, P, P, u32]
        lib.oracle_cost.restype = i64
        lib.oracle_cost.argtypes = [i32, P, P, i64, i32, i32, P, P, P, P]
        lib.oracle_check_full.restype = i64
        lib.oracle_check_full.argtypes = [i32, P, P, i64, i32, i32, P, P, P, P, u32, i64]
        lib.oracle_ls.restype = ctypes.c_int
        lib.oracle_ls.argtypes = [i32, P, P, i64, i32, i32, P, P, u32, i32, i32, P, P, P]
        lib.oracle_eval_pen.restype = ctypes.c_int
        lib.oracle_eval_pen.argtypes = [i32, P, P, i64, i32, i32, P, P, u32, i64, i64, i32, P, P, P, P, P]
        lib.oracle_ls_pen.restype = ctypes.c_int
        lib.oracle_ls_pen.argtypes = [i32, P, P, i64, i32, i32, P, P, u32, i64, i64, i32, i32, P, P, P]
        lib.oracle_granular_mask.restype = None
        lib.oracle_granular_mask.argtypes = [i32, P, i32, P]
        lib.oracle_eval_gran.restype = ctypes.c_int
        lib.oracle_eval_gran.argtypes = [i32, P, P, i64, i32, i32, P, P, u32, P, i32, P, P, P, P, P]
        lib.oracle_ls_gran.restype = ctypes.c_int
        lib.oracle_ls_gran.argtypes = [i32, P, P, i64, i32, i32, P, P, u32, P, i32, i32, P, P, P]
        lib.oracle_violations.restype = None
        lib.oracle_violations.argtypes = [i32, P, P, P, i64, i32, i32, P, P, P, P]
        lib.oracle_eval_ex.restype = ctypes.c_int
        lib.oracle_eval_ex.argtypes = [i32, P, P, P, i64, i32, i32, P, P, u32, P, i32, i64, i64, i32, P, P, P, P, P]
        lib.oracle_ls_ex.restype = ctypes.c_int
        lib.oracle_ls_ex.argtypes = [i32, P, P, P, i64, i32, i32, P, P, u32, P, i32, i64, i64, i32, i32, P, P, P]
        lib.oracle_multi_select.restype = ctypes.c_int
        lib.oracle_multi_select.argtypes = [i32, P, P, P, i64, i32, i32, P, P, u32, i32, i64, i64, i32, i32, P, P,
                                            P, P]
        lib.oracle_ls_multi.restype = ctypes.c_int
        lib.oracle_ls_multi.argtypes = [i32, P, P, P, i64, i32, i32, P, P, u32, i32, i64, i64, i32, i32, i32, P, P,
                                        P, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pickups(inst):
    """Pickup amounts per node (VRPSPDTW), or None."""
    p = getattr(inst, "pickup", None)
    return None if p is None else np.ascontiguousarray(p, dtype=np.int32)


def _inst_args(inst):
    D = np.ascontiguousarray(inst.dist, dtype=np.int32)
    nd = np.ascontiguousarray(inst.node4, dtype=np.int32)
    return D, nd


@dataclass
class Best:
    found: bool
    delta: int
    id: int
    moves: int


def granular_mask(inst, theta: int) -> np.ndarray:
    """(n+1) x (n+1) uint8 pair mask of granular mode: {i, j} is kept when
    either node is among the theta closest to the other."""
    lib = _load()
    D = np.ascontiguousarray(inst.dist, dtype=np.int32)
    m = np.zeros((inst.n + 1, inst.n + 1), np.uint8)
    lib.oracle_granular_mask(inst.n, _p(D), int(theta), _p(m))
    return m


def eval_neighbourhood(inst, sol, op_mask: int = OPS_ALL, threads: int = 0,
                       dump: bool = False, penalty=None, theta=None, mask=None):
    """Best admissible move of N(S) (and, with dump=True, per-move delta and
    feasibility arrays indexed by move id; non-moves keep delta 0 and feas
    0xFF).  penalty=(w_load, w_tw): penalised mode, where every move is
    admissible and `delta` is the score dD + w_load dL_V + w_tw dT_V.
    theta (or a prebuilt granular mask): granular mode, the inter-route
    moves restricted to the granular pairs."""
    lib = _load()
    D, nd = _inst_args(inst)
    off = np.ascontiguousarray(sol.offsets, dtype=np.int32)
    cust = np.ascontiguousarray(sol.customers, dtype=np.int32)
    Q = inst.n + off.shape[0] - 1
    dd = df = None
    if dump:
        span = id_span(op_mask) * Q * Q
        dd = np.zeros(span, np.int32)
        df = np.full(span, NOT_A_MOVE, np.uint8)
    bd = np.zeros(1, np.int64)
    bid = np.zeros(1, np.uint32)
    mv = np.zeros(1, np.int64)
    if theta is not None and mask is None:
        mask = granular_mask(inst, theta)
    pick = _pickups(inst)
    if pick is not None:
        pen = penalty if penalty is not None else (0, 0)
        found = lib.oracle_eval_ex(inst.n, _p(D), _p(nd), _p(pick), inst.capacity, inst.has_tw,
                                   off.shape[0] - 1, _p(off), _p(cust), op_mask,
                                   _p(mask) if mask is not None else None, int(penalty is not None),
                                   int(pen[0]), int(pen[1]), threads,
                                   _p(dd) if dump else None, _p(df) if dump else None,
                                   _p(bd), _p(bid), _p(mv))
    elif mask is not None:
        assert penalty is None
        found = lib.oracle_eval_gran(inst.n, _p(D), _p(nd), inst.capacity, inst.has_tw,
                                     off.shape[0] - 1, _p(off), _p(cust), op_mask, _p(mask), threads,
                                     _p(dd) if dump else None, _p(df) if dump else None,
                                     _p(bd), _p(bid), _p(mv))
    elif penalty is None:
        found = lib.oracle_eval(inst.n, _p(D), _p(nd), inst.capacity, inst.has_tw,
                                off.shape[0] - 1, _p(off), _p(cust), op_mask, threads,
                                _p(dd) if dump else None, _p(df) if dump else None,
                                _p(bd), _p(bid), _p(mv))
    else:
        found = lib.oracle_eval_pen(inst.n, _p(D), _p(nd), inst.capacity, inst.has_tw,
                                    off.shape[0] - 1, _p(off), _p(cust), op_mask,
                                    int(penalty[0]), int(penalty[1]), threads,
                                    _p(dd) if dump else None, _p(df) if dump else None,
                                    _p(bd), _p(bid), _p(mv))
    best = Best(bool(found), int(bd[0]), int(bid[0]), int(mv[0]))
    if dump:
        return best, dd, df
    return best


class Routes:
    """Routes in CSR form (offsets[R+1], customers[n])."""

    def __init__(self, offsets, customers):
        self.offsets = np.asarray(offsets, dtype=np.int32)
        self.customers = np.asarray(customers, dtype=np.int32)

    @property
    def R(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def routes(self):
        o = self.offsets
        return [self.customers[o[r]:o[r + 1]].tolist() for r in range(self.R)]


def apply_move(inst, sol, move_id: int):
    """New routes after applying move_id; raises ValueError for a non-move."""
    lib = _load()
    D, nd = _inst_args(inst)
    off = np.array(sol.offsets, dtype=np.int32)
    cust = np.array(sol.customers, dtype=np.int32)
    rc = lib.oracle_apply(inst.n, _p(D), _p(nd), inst.capacity, inst.has_tw,
                          off.shape[0] - 1, _p(off), _p(cust), move_id)
    if rc != 0:
        raise ValueError("not a move of N(S): %d" % move_id)
    return Routes(off, cust)


def cost(inst, sol):
    """(total distance, #capacity-violating routes, #window-violating routes);
    the counts ignore pickups (use violations() for VRPSPDTW)."""
    lib = _load()
    D, nd = _inst_args(inst)
    off = np.ascontiguousarray(sol.offsets, dtype=np.int32)
    cust = np.ascontiguousarray(sol.customers, dtype=np.int32)
    cb = np.zeros(1, np.int32)
    tb = np.zeros(1, np.int32)
    c = lib.oracle_cost(inst.n, _p(D), _p(nd), inst.capacity, inst.has_tw,
                        off.shape[0] - 1, _p(off), _p(cust), _p(cb), _p(tb))
    return int(c), int(cb[0]), int(tb[0])


def check_full(inst, sol, dump_delta, dump_feas, op_mask: int = OPS_ALL,
               sample_every: int = 1) -> int:
    """Number of moves whose delta differs from a whole-solution recompute."""
    lib = _load()
    D, nd = _inst_args(inst)
    off = np.ascontiguousarray(sol.offsets, dtype=np.int32)
    cust = np.ascontiguousarray(sol.customers, dtype=np.int32)
    return int(lib.oracle_check_full(inst.n, _p(D), _p(nd), inst.capacity, inst.has_tw,
                                     off.shape[0] - 1, _p(off), _p(cust), _p(dump_delta),
                                     _p(dump_feas), op_mask, sample_every))


def violations(inst, sol):
    """(total load excess, total time warp) of S (penalised mode's terms)."""
    lib = _load()
    D, nd = _inst_args(inst)
    off = np.ascontiguousarray(sol.offsets, dtype=np.int32)
    cust = np.ascontiguousarray(sol.customers, dtype=np.int32)
    lv = np.zeros(1, np.int64)
    tv = np.zeros(1, np.int64)
    pick = _pickups(inst)
    lib.oracle_violations(inst.n, _p(D), _p(nd), _p(pick) if pick is not None else None, inst.capacity,
                          inst.has_tw, off.shape[0] - 1, _p(off), _p(cust), _p(lv), _p(tv))
    return int(lv[0]), int(tv[0])


def local_search(inst, sol, op_mask: int = OPS_ALL, max_steps: int = 100,
                 threads: int = 0, penalty=None, theta=None, mask=None):
    """Best-improvement local search.  Returns (final Solution, ids, deltas,
    total moves evaluated).  penalty=(w_load, w_tw): penalised mode (deltas
    are then scores); theta / mask: granular mode."""
    lib = _load()
    D, nd = _inst_args(inst)
    off = np.array(sol.offsets, dtype=np.int32)
    cust = np.array(sol.customers, dtype=np.int32)
    ids = np.zeros(max(1, max_steps), np.uint32)
    deltas = np.zeros(max(1, max_steps), np.int32)
    mv = np.zeros(1, np.int64)
    if theta is not None and mask is None:
        mask = granular_mask(inst, theta)
    pick = _pickups(inst)
    if pick is not None:
        pen = penalty if penalty is not None else (0, 0)
        steps = lib.oracle_ls_ex(inst.n, _p(D), _p(nd), _p(pick), inst.capacity, inst.has_tw,
                                 off.shape[0] - 1, _p(off), _p(cust), op_mask,
                                 _p(mask) if mask is not None else None, int(penalty is not None),
                                 int(pen[0]), int(pen[1]), max_steps, threads, _p(ids), _p(deltas), _p(mv))
    elif mask is not None:
        assert penalty is None
        steps = lib.oracle_ls_gran(inst.n, _p(D), _p(nd), inst.capacity, inst.has_tw,
                                   off.shape[0] - 1, _p(off), _p(cust), op_mask, _p(mask), max_steps,
                                   threads, _p(ids), _p(deltas), _p(mv))
    elif penalty is None:
        steps = lib.oracle_ls(inst.n, _p(D), _p(nd), inst.capacity, inst.has_tw,
                              off.shape[0] - 1, _p(off), _p(cust), op_mask, max_steps, threads,
                              _p(ids), _p(deltas), _p(mv))
    else:
        steps = lib.oracle_ls_pen(inst.n, _p(D), _p(nd), inst.capacity, inst.has_tw,
                                  off.shape[0] - 1, _p(off), _p(cust), op_mask, int(penalty[0]),
                                  int(penalty[1]), max_steps, threads, _p(ids), _p(deltas), _p(mv))
    return Routes(off, cust), ids[:steps].copy(), deltas[:steps].copy(), int(mv[0])


def multi_select(inst, sol, op_mask: int = OPS_ALL, threads: int = 0, penalty=None, candidates=False):
    """Independent moves of one multi-move step (Section 7): per pair of
    route slots the best admissible improving move touching exactly those
    routes, then taken greedily in (delta, id) order when its routes are
    still free.  Returns ([(id, delta)] in selection order, |N(S)|), and
    with candidates=True also the number of route pairs with a candidate."""
    lib = _load()
    D, nd = _inst_args(inst)
    off = np.ascontiguousarray(sol.offsets, dtype=np.int32)
    cust = np.ascontiguousarray(sol.customers, dtype=np.int32)
    R = off.shape[0] - 1
    ids = np.zeros(R, np.uint32)
    dl = np.zeros(R, np.int64)
    mv = np.zeros(1, np.int64)
    nc = np.zeros(1, np.int64)
    pick = _pickups(inst)
    pen = penalty if penalty is not None else (0, 0)
    cnt = lib.oracle_multi_select(inst.n, _p(D), _p(nd), _p(pick) if pick is not None else None, inst.capacity,
                                  inst.has_tw, R, _p(off), _p(cust), op_mask, int(penalty is not None),
                                  int(pen[0]), int(pen[1]), threads, R, _p(ids), _p(dl), _p(mv), _p(nc))
    sel = [(int(ids[q]), int(dl[q])) for q in range(cnt)]
    return (sel, int(mv[0]), int(nc[0])) if candidates else (sel, int(mv[0]))


def local_search_multi(inst, sol, op_mask: int = OPS_ALL, max_steps: int = 100, threads: int = 0,
                       penalty=None):
    """Multi-move local search: repeat {multi_select; apply the selection in
    order} while something is selected, at most max_steps steps.  Returns
    (final Routes, [(id, delta)] applied in order, moves per step, total
    moves evaluated)."""
    lib = _load()
    D, nd = _inst_args(inst)
    off = np.array(sol.offsets, dtype=np.int32)
    cust = np.array(sol.customers, dtype=np.int32)
    R = off.shape[0] - 1
    cap = max(1, max_steps) * R
    ids = np.zeros(cap, np.uint32)
    dl = np.zeros(cap, np.int32)
    per = np.zeros(max(1, max_steps), np.int32)
    mv = np.zeros(1, np.int64)
    pick = _pickups(inst)
    pen = penalty if penalty is not None else (0, 0)
    it = lib.oracle_ls_multi(inst.n, _p(D), _p(nd), _p(pick) if pick is not None else None, inst.capacity,
                             inst.has_tw, R, _p(off), _p(cust), op_mask, int(penalty is not None), int(pen[0]),
                             int(pen[1]), max_steps, threads, cap, _p(ids), _p(dl), _p(per), _p(mv))
    nm = int(per[:it].sum())
    return Routes(off, cust), [(int(ids[q]), int(dl[q])) for q in range(nm)], per[:it].tolist(), int(mv[0])


def decode(Q: int, move_id: int):
    """(op, k, a, b) of a move id."""
    qq = Q * Q
    opk, rem = divmod(int(move_id), qq)
    return opk // 4, opk % 4, rem // Q, rem % Q
