"""Python binding of the C ABI in include/tga.h (argument marshalling only).

PyTorch provides device memory (int32 / uint8 tensors on ``cuda``) and the
stream (``torch.cuda.current_stream().cuda_stream``); every step of the path
runs in the HIP kernels of ``libtga.so``.  There is no fallback: if the
library is missing or fails to load, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtga.so")

TGA_OK, TGA_ENOMOVE = 0, 1
TGA_EINVAL, TGA_ERANGE, TGA_ENOMEM, TGA_EDEVICE, TGA_ESTALE = -1, -2, -3, -4, -5
OP_RELOCATE, OP_SWAP, OP_2OPTSTAR, OP_2OPT, OP_OROPT = 1, 2, 4, 8, 16
OPS_ALL = 0x1F
OP_SEGREL, OP_SEGREL_REV, OP_CROSS = 1 << 5, 1 << 6, 1 << 7  # operator variants (general path)
OPS_VARIANTS = 0xE0
OP_GRANULAR = 1 << 16  # modifier: inter-route operators on the granular pairs only
OP_COUNT_FULL = 1 << 17  # modifier (batched local search): count the pairs evaluated in full
OP_MULTI = 1 << 18  # modifier (general path): several independent moves per local-search step
MAX_Q = 14654

_lib = None


class TGAError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("tga error %d: %s" % (code, msg))
        self.code = code


class Move(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("k", ctypes.c_int32), ("a", ctypes.c_int32),
                ("b", ctypes.c_int32), ("delta", ctypes.c_int32), ("feas", ctypes.c_uint32),
                ("id", ctypes.c_uint32), ("version", ctypes.c_uint32)]

    def __repr__(self):
        return ("Move(op=%d, k=%d, a=%d, b=%d, delta=%d, feas=%d, id=%d, version=%d)"
                % (self.op, self.k, self.a, self.b, self.delta, self.feas, self.id, self.version))


class BatchConfig(ctypes.Structure):
    """Schedule of a batch (tga_batch_config_t); never changes a result."""
    _fields_ = [("lds_kb", ctypes.c_int32), ("split", ctypes.c_int32), ("rows_per_item", ctypes.c_int32),
                ("sub_rows", ctypes.c_int32), ("us_per_eval", ctypes.c_float)]

    def as_dict(self):
        return {"lds_kb": self.lds_kb, "split": self.split, "rows_per_item": self.rows_per_item,
                "sub_rows": self.sub_rows, "us_per_eval": round(float(self.us_per_eval), 2)}


class TuneEntry(ctypes.Structure):
    """One row of the schedule table (tga_tune_entry_t)."""
    _fields_ = [("has_tw", ctypes.c_int32), ("n_max", ctypes.c_int32), ("plain_rows", ctypes.c_int32),
                ("item_rows", ctypes.c_int32)]


# The schedule table the autotuner (paper_2506_17357_amd/autotune.py) writes;
# applied when the library is loaded.  TGA_TUNE_TABLE names another file ("" = none).
TUNE_PATH = os.environ.get("TGA_TUNE_TABLE", os.path.join(HERE, "tune_table.json"))

EXPORTS = [
    "tga_instance_workspace_bytes", "tga_solution_workspace_bytes", "tga_load_instance",
    "tga_set_solution", "tga_eval_neighborhood", "tga_apply_move", "tga_ls_run",
    "tga_get_solution", "tga_move_counts", "tga_solution_version", "tga_free_solution",
    "tga_free_instance", "tga_last_error", "tga_batch_workspace_bytes", "tga_batch_create",
    "tga_batch_ls_run", "tga_batch_eval", "tga_batch_reset", "tga_batch_free",
    "tga_device_limits", "tga_batch_begin", "tga_batch_step_part", "tga_batch_collect",
    "tga_solution_reload", "tga_solution_begin", "tga_batch_poll", "tga_solution_stats",
    "tga_instance_dist_bytes", "tga_batch_get_config", "tga_batch_set_config", "tga_batch_autotune",
    "tga_eval_routes_static", "tga_batch_slots_workspace_bytes", "tga_batch_create_slots",
    "tga_batch_set_members", "tga_batch_tick", "tga_batch_tick_status",
    "tga_granular_workspace_bytes", "tga_instance_set_granular", "tga_instance_granular_pairs",
    "tga_solution_set_penalty", "tga_solution_violations", "tga_instance_set_pickups",
    "tga_solution_set_general", "tga_solution_screen_stats", "tga_batch_screen_stats",
    "tga_set_tuning", "tga_solution_set_rows", "tga_solution_get_rows", "tga_probe_stream_read",
    "tga_multi_workspace_bytes", "tga_solution_set_multi", "tga_solution_select_moves", "tga_solution_multi_stats",
]


def lib():
    """Load libtga.so (raises if it is missing: there is no other path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libtga.so is not built (run __graft_entry__.build() or "
                           "python paper_2506_17357_amd/build_lib.py)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "tga_instance_workspace_bytes": (sz, [i32]),
        "tga_solution_workspace_bytes": (sz, [i32, i32]),
        "tga_load_instance": (i32, [i32, P, P, i32, i32, P, sz, P, pp]),
        "tga_set_solution": (i32, [P, i32, P, P, P, sz, P, pp]),
        "tga_eval_neighborhood": (i32, [P, u32, ctypes.POINTER(Move), P, P, P]),
        "tga_eval_routes_static": (i32, [P, i32, P, P, u32, ctypes.POINTER(Move), P]),
        "tga_batch_slots_workspace_bytes": (sz, [i32, i32, i32]),
        "tga_granular_workspace_bytes": (sz, [i32, i32]),
        "tga_solution_set_penalty": (i32, [P, i32, i32, P]),
        "tga_instance_set_pickups": (i32, [P, P, P]),
        "tga_solution_set_general": (i32, [P, i32, P]),
        "tga_solution_screen_stats": (i32, [P, P, P]),
        "tga_batch_screen_stats": (i32, [P, P, P]),
        "tga_set_tuning": (i32, [P, i32]),
        "tga_probe_stream_read": (i32, [P, sz, P]),
        "tga_multi_workspace_bytes": (sz, [i32]),
        "tga_solution_set_multi": (i32, [P, P, sz, P]),
        "tga_solution_select_moves": (i32, [P, ctypes.POINTER(Move), i32, P, P]),
        "tga_solution_multi_stats": (i32, [P, P, P]),
        "tga_solution_set_rows": (i32, [P, i32, i32, P]),
        "tga_solution_get_rows": (i32, [P, P, P]),
        "tga_solution_violations": (i32, [P, P, P, P]),
        "tga_instance_set_granular": (i32, [P, i32, P, sz, P]),
        "tga_instance_granular_pairs": (i32, [P]),
        "tga_batch_create_slots": (i32, [i32, i32, i32, P, sz, P, pp]),
        "tga_batch_set_members": (i32, [P, P, P]),
        "tga_batch_tick": (i32, [P, u32, i32, P, P]),
        "tga_batch_tick_status": (i32, [P, P, P, P, P, P]),
        "tga_apply_move": (i32, [P, ctypes.POINTER(Move), P, P]),
        "tga_ls_run": (i32, [P, u32, i32, P, P, P, P]),
        "tga_get_solution": (i32, [P, P, P, P, P]),
        "tga_move_counts": (i32, [P, P, P]),
        "tga_solution_version": (u32, [P]),
        "tga_free_solution": (i32, [P]),
        "tga_free_instance": (i32, [P]),
        "tga_last_error": (ctypes.c_char_p, []),
        "tga_batch_workspace_bytes": (sz, [P, i32]),
        "tga_batch_create": (i32, [P, i32, i32, i32, P, sz, P, pp]),
        "tga_batch_ls_run": (i32, [P, u32, i32, i32, P, P, P, P]),
        "tga_batch_eval": (i32, [P, u32, ctypes.POINTER(Move), P, P]),
        "tga_batch_reset": (i32, [P, P]),
        "tga_batch_free": (i32, [P]),
        "tga_device_limits": (i32, [P, P]),
        "tga_batch_begin": (i32, [P, i32, P]),
        "tga_batch_step_part": (i32, [P, u32, i32, P]),
        "tga_batch_collect": (i32, [P, P, P, P, P]),
        "tga_solution_reload": (i32, [P, P, P, P]),
        "tga_solution_begin": (i32, [P, i32, P]),
        "tga_batch_poll": (i32, [P, P, P]),
        "tga_solution_stats": (i32, [P, P, P, P, P, P]),
        "tga_instance_dist_bytes": (i32, [P]),
        "tga_batch_get_config": (i32, [P, ctypes.POINTER(BatchConfig)]),
        "tga_batch_set_config": (i32, [P, ctypes.POINTER(BatchConfig), P]),
        "tga_batch_autotune": (i32, [P, u32, i32, ctypes.POINTER(BatchConfig), P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    if TUNE_PATH and os.path.exists(TUNE_PATH):
        load_tuning(TUNE_PATH)
    return L


def set_tuning(entries):
    """Install a schedule table: entries of dicts with kind ("cvrp" or
    "vrptw"), n_max, plain_rows, item_rows (tga_set_tuning)."""
    arr = (TuneEntry * max(1, len(entries)))()
    for k, e in enumerate(entries):
        arr[k] = TuneEntry(int(e["kind"] != "cvrp"), int(e["n_max"]), int(e["plain_rows"]), int(e["item_rows"]))
    _check(lib().tga_set_tuning(arr, len(entries)))


def load_tuning(path: str):
    """Install the table of a JSON file written by the autotuner."""
    import json
    with open(path) as f:
        set_tuning(json.load(f)["entries"])


def _check(rc: int, allow=(TGA_OK,)):
    if rc in allow:
        return rc
    raise TGAError(rc, lib().tga_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dev_ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Instance:
    """Device-resident instance: distance matrix and node data."""

    def __init__(self, n: int, dist, node4, capacity: int, has_tw: int, device="cuda", stream=None):
        L = lib()
        self.n = int(n)
        self.dist = torch.as_tensor(np.ascontiguousarray(dist, dtype=np.int32)).to(device) \
            if not isinstance(dist, torch.Tensor) else dist
        self.node4 = torch.as_tensor(np.ascontiguousarray(node4, dtype=np.int32)).to(device) \
            if not isinstance(node4, torch.Tensor) else node4
        self.capacity = int(capacity)
        self.has_tw = int(has_tw)
        nbytes = L.tga_instance_workspace_bytes(self.n)
        if nbytes == 0:
            raise TGAError(TGA_ERANGE, "n = %d out of range" % n)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(L.tga_load_instance(self.n, _dev_ptr(self.dist), _dev_ptr(self.node4), self.capacity,
                                   self.has_tw, _dev_ptr(self.ws), nbytes, _stream(stream),
                                   ctypes.byref(h)))
        self.h = h

    def set_granular(self, theta: int, stream=None):
        """Granular pairs of the theta nearest neighbours (edge-based
        neighbourhood reduction); evaluations then accept OP_GRANULAR."""
        L = lib()
        nbytes = L.tga_granular_workspace_bytes(self.n, int(theta))
        if nbytes == 0:
            raise TGAError(TGA_ERANGE, "theta = %d out of range" % theta)
        self.gws = torch.empty(nbytes, dtype=torch.uint8, device=self.dist.device)
        _check(L.tga_instance_set_granular(self.h, int(theta), _dev_ptr(self.gws), nbytes, _stream(stream)))
        self.theta = int(theta)

    @property
    def granular_pairs(self) -> int:
        return int(lib().tga_instance_granular_pairs(self.h))

    @property
    def dist_bytes(self) -> int:
        """Bytes per distance the inter-route kernels stream (2 or 4)."""
        return int(lib().tga_instance_dist_bytes(self.h))

    def set_pickups(self, pickup, stream=None):
        """Pickup amount per node (VRPSPDTW); solutions set up afterwards use it."""
        self.pickup = torch.as_tensor(np.ascontiguousarray(pickup, dtype=np.int32)).to(self.dist.device) \
            if not isinstance(pickup, torch.Tensor) else pickup
        _check(lib().tga_instance_set_pickups(self.h, _dev_ptr(self.pickup), _stream(stream)))

    @staticmethod
    def from_workload(inst, device="cuda", stream=None) -> "Instance":
        I = Instance(inst.n, inst.dist, inst.node4, inst.capacity, inst.has_tw, device, stream)
        if getattr(inst, "pickup", None) is not None:
            I.set_pickups(inst.pickup, stream)
        return I

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tga_free_instance(self.h)
            self.h = None


class Solution:
    """A solution held on the device with its attribute arrays."""

    def __init__(self, inst: Instance, offsets, customers, stream=None):
        L = lib()
        self.inst = inst
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        cust = np.ascontiguousarray(customers, dtype=np.int32)
        self.R = int(off.shape[0] - 1)
        self.Q = inst.n + self.R
        nbytes = L.tga_solution_workspace_bytes(inst.n, self.R)
        if nbytes == 0:
            raise TGAError(TGA_ERANGE, "n + R = %d out of range" % self.Q)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=inst.dist.device)
        h = ctypes.c_void_p()
        _check(L.tga_set_solution(inst.h, self.R, _np_ptr(off), _np_ptr(cust), _dev_ptr(self.ws),
                                  nbytes, _stream(stream), ctypes.byref(h)))
        self.h = h

    def reload(self, offsets, customers, stream=None):
        """Replace the routes in place (same workspace; batches stay valid)."""
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        cust = np.ascontiguousarray(customers, dtype=np.int32)
        _check(lib().tga_solution_reload(self.h, _np_ptr(off), _np_ptr(cust), _stream(stream)))

    def set_penalty(self, w_load: int, w_tw: int = 0, stream=None):
        """Penalised scoring dD + w_load dL_V + w_tw dT_V (every move
        admissible); w_load < 0 returns to hard feasibility."""
        _check(lib().tga_solution_set_penalty(self.h, int(w_load), int(w_tw), _stream(stream)))

    def set_general(self, on: bool = True, stream=None):
        """Evaluate through the general (concatenation) path, which the
        operator variants need."""
        _check(lib().tga_solution_set_general(self.h, int(bool(on)), _stream(stream)))

    def violations(self, stream=None):
        """(total load excess, total time warp) in penalised mode."""
        lv = ctypes.c_int64()
        tv = ctypes.c_int64()
        _check(lib().tga_solution_violations(self.h, ctypes.byref(lv), ctypes.byref(tv), _stream(stream)))
        return int(lv.value), int(tv.value)

    def begin(self, max_steps: int, stream=None):
        """Clear counters and set the step cap before joining a running batch."""
        _check(lib().tga_solution_begin(self.h, max_steps, _stream(stream)))

    def eval(self, op_mask: int = OPS_ALL, dump: bool = False, stream=None):
        """Best admissible move (or None); with dump=True also the per-move
        delta / feasibility tensors (non-moves keep 0 / 0xFF)."""
        L = lib()
        m = Move()
        dd = df = None
        if dump:
            size = (40 if op_mask & OPS_VARIANTS else 20) * self.Q * self.Q
            dd = torch.zeros(size, dtype=torch.int32, device=self.ws.device)
            df = torch.full((size,), 0xFF, dtype=torch.uint8, device=self.ws.device)
        rc = _check(L.tga_eval_neighborhood(self.h, op_mask, ctypes.byref(m),
                                            _dev_ptr(dd) if dump else None,
                                            _dev_ptr(df) if dump else None, _stream(stream)),
                    allow=(TGA_OK, TGA_ENOMOVE))
        best = None if rc == TGA_ENOMOVE else m
        if dump:
            return best, dd, df
        return best

    def apply(self, move: Move, stream=None) -> int:
        cost = ctypes.c_int64()
        _check(lib().tga_apply_move(self.h, ctypes.byref(move), ctypes.byref(cost), _stream(stream)))
        return int(cost.value)

    def ls_run(self, max_steps: int, op_mask: int = OPS_ALL, stream=None):
        """Device-resident local search; returns (steps, moves evaluated, cost)."""
        steps = ctypes.c_int32()
        mv = ctypes.c_int64()
        cost = ctypes.c_int64()
        _check(lib().tga_ls_run(self.h, op_mask, max_steps, ctypes.byref(steps), ctypes.byref(mv),
                                ctypes.byref(cost), _stream(stream)))
        return int(steps.value), int(mv.value), int(cost.value)

    def get(self, stream=None):
        """(offsets, customers, cost) of the current solution."""
        off = np.zeros(self.R + 1, np.int32)
        cust = np.zeros(self.inst.n, np.int32)
        cost = ctypes.c_int64()
        _check(lib().tga_get_solution(self.h, _np_ptr(off), _np_ptr(cust), ctypes.byref(cost),
                                      _stream(stream)))
        return off, cust, int(cost.value)

    def stats(self, stream=None):
        """(accepted moves, converged, moves evaluated, cost) since the last begin/ls_run."""
        st = ctypes.c_int32()
        cv = ctypes.c_int32()
        mv = ctypes.c_int64()
        cost = ctypes.c_int64()
        _check(lib().tga_solution_stats(self.h, ctypes.byref(st), ctypes.byref(cv), ctypes.byref(mv),
                                        ctypes.byref(cost), _stream(stream)))
        return int(st.value), bool(cv.value), int(mv.value), int(cost.value)

    def set_multi(self, on: bool = True, stream=None):
        """Multi-move local search (OP_MULTI): allocates the per-route-pair
        table on the solution's device, or drops it."""
        if on:
            nb = int(lib().tga_multi_workspace_bytes(self.R))
            self._multi_ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.ws.device)
            base = self._multi_ws.data_ptr()
            ptr = (base + 255) // 256 * 256
            _check(lib().tga_solution_set_multi(self.h, ctypes.c_void_p(ptr), nb, _stream(stream)))
        else:
            _check(lib().tga_solution_set_multi(self.h, None, 0, _stream(stream)))
            self._multi_ws = None

    def select_moves(self, stream=None):
        """The independent moves selected from the table the last
        eval(op_mask | OP_MULTI) filled, in selection order (not applied)."""
        cap = self.R
        arr = (Move * cap)()
        cnt = ctypes.c_int32()
        _check(lib().tga_solution_select_moves(self.h, arr, cap, ctypes.byref(cnt), _stream(stream)))
        return list(arr[:cnt.value])

    def multi_stats(self, stream=None):
        """(steps, moves applied) of the last multi-move tga_ls_run."""
        c = np.zeros(2, np.int64)
        _check(lib().tga_solution_multi_stats(self.h, _np_ptr(c), _stream(stream)))
        return int(c[0]), int(c[1])

    def set_rows(self, plain_rows: int = 0, item_rows: int = 0, stream=None):
        """Schedule of this solution (tga_solution_set_rows; 0 = table / default)."""
        _check(lib().tga_solution_set_rows(self.h, int(plain_rows), int(item_rows), _stream(stream)))

    def rows(self):
        """(rows per item of the single-solution form, of the batched form; 0 = default rule)."""
        a = ctypes.c_int32()
        b = ctypes.c_int32()
        _check(lib().tga_solution_get_rows(self.h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def screen_stats(self, stream=None):
        """(pairs evaluated in full, pairs visited) by the inter-route
        screens of the local-search evaluations since the last reset."""
        c = np.zeros(2, np.int64)
        _check(lib().tga_solution_screen_stats(self.h, _np_ptr(c), _stream(stream)))
        return int(c[0]), int(c[1])

    def move_counts(self, stream=None) -> np.ndarray:
        c = np.zeros(5, np.int64)
        _check(lib().tga_move_counts(self.h, _np_ptr(c), _stream(stream)))
        return c

    @property
    def version(self) -> int:
        return int(lib().tga_solution_version(self.h))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tga_free_solution(self.h)
            self.h = None


class Batch:
    """Many solutions stepped together by one persistent launch per step."""

    def __init__(self, sols: list[Solution], rows_per_item: int = 0, sub_rows: int = 0, stream=None):
        L = lib()
        self.sols = list(sols)
        arr = (ctypes.c_void_p * len(self.sols))(*[s.h.value for s in self.sols])
        self._arr = arr
        nbytes = L.tga_batch_workspace_bytes(arr, len(self.sols))
        if nbytes == 0:
            raise TGAError(TGA_EINVAL, "bad batch")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.sols[0].ws.device)
        h = ctypes.c_void_p()
        _check(L.tga_batch_create(arr, len(self.sols), rows_per_item, sub_rows, _dev_ptr(self.ws),
                                  nbytes, _stream(stream), ctypes.byref(h)))
        self.h = h

    def ls_run(self, steps: int, op_mask: int = OPS_ALL, use_graph: bool = True, stream=None):
        n = len(self.sols)
        st = np.zeros(n, np.int32)
        mv = np.zeros(n, np.int64)
        cost = np.zeros(n, np.int64)
        _check(lib().tga_batch_ls_run(self.h, op_mask, steps, int(use_graph), _np_ptr(st),
                                      _np_ptr(mv), _np_ptr(cost), _stream(stream)))
        return st, mv, cost

    def begin(self, max_steps: int, stream=None):
        _check(lib().tga_batch_begin(self.h, max_steps, _stream(stream)))

    def config(self) -> dict:
        c = BatchConfig()
        _check(lib().tga_batch_get_config(self.h, ctypes.byref(c)))
        return c.as_dict()

    def set_config(self, lds_kb: int, split: int, rows_per_item: int = 0, sub_rows: int = 0, stream=None):
        c = BatchConfig(lds_kb, split, rows_per_item, sub_rows, 0.0)
        _check(lib().tga_batch_set_config(self.h, ctypes.byref(c), _stream(stream)))

    def autotune(self, op_mask: int = OPS_ALL, launches: int = 5, stream=None) -> dict:
        """Pick the fastest schedule for the batch's current state (see
        tga_batch_autotune); returns it."""
        c = BatchConfig()
        _check(lib().tga_batch_autotune(self.h, op_mask, launches, ctypes.byref(c), _stream(stream)))
        return c.as_dict()

    def step_part(self, part: int, op_mask: int = OPS_ALL, stream=None):
        _check(lib().tga_batch_step_part(self.h, op_mask, part, _stream(stream)))

    def collect(self, stream=None):
        n = len(self.sols)
        st = np.zeros(n, np.int32)
        mv = np.zeros(n, np.int64)
        cost = np.zeros(n, np.int64)
        _check(lib().tga_batch_collect(self.h, _np_ptr(st), _np_ptr(mv), _np_ptr(cost), _stream(stream)))
        return st, mv, cost

    def poll(self, stream=None) -> np.ndarray:
        """Converged flag per solution (one device gather + one copy)."""
        d = np.zeros(len(self.sols), np.int32)
        _check(lib().tga_batch_poll(self.h, _np_ptr(d), _stream(stream)))
        return d

    def eval(self, op_mask: int = OPS_ALL, stream=None):
        n = len(self.sols)
        moves = (Move * n)()
        status = np.zeros(n, np.int32)
        _check(lib().tga_batch_eval(self.h, op_mask, moves, _np_ptr(status), _stream(stream)))
        return list(moves), status

    def reset(self, stream=None):
        _check(lib().tga_batch_reset(self.h, _stream(stream)))

    def screen_stats(self, stream=None):
        """The solutions' screening counters summed (see Solution.screen_stats)."""
        c = np.zeros(2, np.int64)
        _check(lib().tga_batch_screen_stats(self.h, _np_ptr(c), _stream(stream)))
        return int(c[0]), int(c[1])

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tga_batch_free(self.h)
            self.h = None

    def __del__(self):
        self.close()


class SlotBatch(Batch):
    """A batch of fixed slots whose members change while it runs (served
    form): asynchronous membership updates and ticks, non-blocking status."""

    def __init__(self, slots: int, max_sum_q: int, max_sum_r: int, device="cuda", stream=None):
        L = lib()
        self.slots = int(slots)
        self.sols = [None] * self.slots
        nbytes = L.tga_batch_slots_workspace_bytes(self.slots, int(max_sum_q), int(max_sum_r))
        if nbytes == 0:
            raise TGAError(TGA_ERANGE, "bad slot batch sizes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(L.tga_batch_create_slots(self.slots, int(max_sum_q), int(max_sum_r), _dev_ptr(self.ws), nbytes,
                                        _stream(stream), ctypes.byref(h)))
        self.h = h
        self._st = np.zeros(self.slots, np.int32)
        self._cv = np.zeros(self.slots, np.int32)
        self._mv = np.zeros(self.slots, np.int64)
        self._cost = np.zeros(self.slots, np.int64)

    def set_members(self, sols, stream=None):
        """sols: one Solution or None per slot."""
        if len(sols) != self.slots:
            raise ValueError("need %d entries" % self.slots)
        arr = (ctypes.c_void_p * self.slots)(*[s.h.value if s is not None else None for s in sols])
        _check(lib().tga_batch_set_members(self.h, arr, _stream(stream)))
        self.sols = list(sols)

    def tick(self, steps: int, op_mask: int = OPS_ALL, stream=None) -> int:
        t = ctypes.c_int32()
        _check(lib().tga_batch_tick(self.h, op_mask, steps, ctypes.byref(t), _stream(stream)))
        return int(t.value)

    def status(self):
        """(tick, converged, steps, moves, cost) of the newest finished tick
        (tick = -1 and no arrays when none has finished)."""
        t = ctypes.c_int32()
        _check(lib().tga_batch_tick_status(self.h, ctypes.byref(t), _np_ptr(self._cv), _np_ptr(self._st),
                                           _np_ptr(self._mv), _np_ptr(self._cost)))
        if t.value < 0:
            return -1, None, None, None, None
        return int(t.value), self._cv.copy(), self._st.copy(), self._mv.copy(), self._cost.copy()


def probe_stream_read(t: torch.Tensor, stream=None):
    """Read a device tensor once through the 16-byte LDS DMA (profiler
    calibration; see tga_probe_stream_read)."""
    _check(lib().tga_probe_stream_read(_dev_ptr(t), t.numel() * t.element_size(), _stream(stream)))


def device_limits():
    """(compute units, LDS bytes per evaluation workgroup)."""
    cu = ctypes.c_int32()
    lds = ctypes.c_int32()
    _check(lib().tga_device_limits(ctypes.byref(cu), ctypes.byref(lds)))
    return int(cu.value), int(lds.value)


STATIC_SCRATCH_BYTES = 8 << 20  # TGA_STATIC_SCRATCH_BYTES


def eval_routes_static(inst: "Instance", offsets, customers, op_mask: int = OPS_ALL, stream=None):
    """Best admissible move (or None) of the given routes, evaluated in the
    library's static per-GPU scratch (tga_eval_routes_static: no workspace,
    nothing allocated)."""
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    cust = np.ascontiguousarray(customers, dtype=np.int32)
    m = Move()
    rc = _check(lib().tga_eval_routes_static(inst.h, int(off.shape[0] - 1), _np_ptr(off), _np_ptr(cust),
                                            op_mask, ctypes.byref(m), _stream(stream)),
                allow=(TGA_OK, TGA_ENOMOVE))
    return None if rc == TGA_ENOMOVE else m
