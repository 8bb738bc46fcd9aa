"""ctypes binding of libsqc (argument marshalling only).

Every function here has the name of the C entry point without the ``sqc_``
prefix and passes plain pointers and sizes through; all computation happens in
the HIP library.  PyTorch supplies device memory (``tensor.data_ptr()``) and
streams (``torch.cuda.current_stream().cuda_stream``).

The library is loaded from this package directory (``libsqc.so``, built by
``paper_2207_00933_amd.build``).  Importing torch first makes the library
resolve the same HIP runtime torch uses.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_size_t, c_uint64, c_void_p
from typing import List, Optional, Sequence

import torch  # noqa: F401  (loads the HIP runtime the library will share)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsqc.so")

OK, E_ARG, E_SHAPE, E_NOMEM, E_DEVICE, E_NUMERIC, E_BUSY, E_UNSUPPORTED = range(8)
MAX_SLICED = 8  # SQC_MAX_SLICED
F64, F32, BF16X3, AUTO = 0, 1, 2, 3
LAYOUT_ATTRIBUTED, LAYOUT_MERGED = 0, 1
MAX_DEGREE = 15
MAX_TOPR = 64
NOALLOC_SCRATCH_BYTES = 64 << 20
STATUS_NAMES = ["SQC_OK", "SQC_E_ARG", "SQC_E_SHAPE", "SQC_E_NOMEM", "SQC_E_DEVICE",
                "SQC_E_NUMERIC", "SQC_E_BUSY", "SQC_E_UNSUPPORTED"]


class Cut(ctypes.Structure):
    _fields_ = [("up_sub", c_int32), ("up_wire", c_int32),
                ("down_sub", c_int32), ("down_wire", c_int32)]


class Sub(ctypes.Structure):
    _fields_ = [("n_wires", c_int32), ("n_data", c_int32), ("data_wire", POINTER(c_int32))]


class Masks(ctypes.Structure):
    _fields_ = [("fixed", c_uint64), ("fixed_val", c_uint64),
                ("active", c_uint64), ("merged", c_uint64)]

    def as_tuple(self):
        return (self.fixed, self.fixed_val, self.active, self.merged)


class Tensor(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("n_labels", c_int32), ("n_bits", c_int32),
                ("prec", c_int), ("layout", c_int32)]


class Cost(ctypes.Structure):
    _fields_ = [("input_floats", c_double), ("plan_mults", c_double),
                ("max_step_operand_floats", c_double), ("max_intermediate_floats", c_double),
                ("naive_mults", c_double), ("n_steps", c_int32), ("order", c_int32 * 128)]


class Found(ctypes.Structure):
    _fields_ = [("prob", c_double), ("recursion", c_int32), ("pad", c_int32), ("bin", c_uint64)]


class RecursionInfo(ctypes.Structure):
    _fields_ = [("bins_sum", c_double), ("parent_prob", c_double), ("top_prob", c_double),
                ("active_bits", c_int32), ("leaf", c_int32)]


class StageTime(ctypes.Structure):
    _fields_ = [("ms", c_double), ("launches", ctypes.c_int64), ("bytes", c_double),
                ("flops", c_double)]


class TuneReport(ctypes.Structure):
    _fields_ = [("steps", c_int32), ("candidates", c_int32), ("default_us", c_double),
                ("tuned_us", c_double), ("step_tile", c_int32 * 64), ("step_groups", c_int32 * 64),
                ("step_nmajor", c_int32 * 64)]


class Request(ctypes.Structure):
    _fields_ = [("circuit", c_int32), ("top_r", c_int32), ("max_bins_M", c_uint64),
                ("scope", POINTER(Masks)), ("prec", c_int), ("bins_prec", c_int),
                ("bins_dev", c_void_p), ("topr_dev", c_void_p), ("sum_dev", c_void_p),
                ("masks_out", POINTER(Masks))]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", c_uint64), ("admitted", c_uint64), ("completed", c_uint64),
                ("running", c_int32), ("queued", c_int32), ("max_running", c_int32),
                ("max_batch", c_int32), ("workspace_bytes", c_uint64), ("workspace_peak", c_uint64),
                ("batches", c_uint64), ("plan_seconds", c_double), ("launch_seconds", c_double),
                ("aged_holds", c_uint64)]


WAITING, RUNNING, DONE = 0, 1, 2

STAGE_ATTRIBUTE, STAGE_MERGE, STAGE_CONTRACT, STAGE_FINAL, STAGE_TOPR = 1, 2, 4, 8, 16


class SqcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2207_00933_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = c_void_p
        sig = {
            "sqc_version": (c_char_p, []),
            "sqc_last_error": (c_char_p, [P]),
            "sqc_ctx_create": (c_int, [c_int, P, POINTER(P)]),
            "sqc_ctx_destroy": (c_int, [P]),
            "sqc_ctx_set_stream": (c_int, [P, P]),
            "sqc_ctx_set_workspace": (c_int, [P, P, c_size_t]),
            "sqc_ctx_set_timing": (c_int, [P, ctypes.c_uint32]),
            "sqc_ctx_timing": (c_int, [P, ctypes.c_uint32, c_int32, POINTER(StageTime)]),
            "sqc_check_graph": (c_int, [POINTER(Sub), c_int32, POINTER(Cut), c_int32]),
            "sqc_assign_bins": (c_int, [c_int32, POINTER(c_int32), POINTER(Masks), c_uint64,
                                        POINTER(Masks)]),
            "sqc_bin_scope": (c_int, [c_int32, POINTER(Masks), c_uint64, POINTER(Masks)]),
            "sqc_plan_cost": (c_int, [c_int32, POINTER(c_int32), POINTER(Cut), c_int32,
                                      POINTER(c_int32), POINTER(Cost)]),
            "sqc_slice_plan": (c_int, [c_int32, POINTER(c_int32), POINTER(Cut), c_int32,
                                       c_double, POINTER(c_int32), POINTER(c_int32)]),
            "sqc_find_cuts": (c_int, [c_int32, POINTER(c_int32), c_int32, c_int32, c_double,
                                      ctypes.c_int64, POINTER(c_int32), POINTER(c_int32),
                                      POINTER(c_int32), POINTER(c_int32)]),
            "sqc_attribute_bytes": (c_size_t, [POINTER(Sub), c_int32, c_int32, POINTER(Cut),
                                               c_int32, c_int]),
            "sqc_attribute": (c_int, [P, POINTER(Sub), c_int32, c_int32, POINTER(Cut), c_int32,
                                      P, c_int, POINTER(Tensor)]),
            "sqc_attribute_all": (c_int, [P, POINTER(Sub), c_int32, POINTER(Cut), c_int32,
                                          POINTER(c_void_p), c_int, POINTER(Tensor)]),
            "sqc_attribute_all_merged": (c_int, [P, POINTER(Sub), c_int32, POINTER(Cut), c_int32,
                                                 POINTER(c_void_p), c_int, POINTER(Tensor)]),
            "sqc_merge_workspace_bytes": (c_size_t, [POINTER(Tensor), POINTER(Masks)]),
            "sqc_merge": (c_int, [P, POINTER(Tensor), POINTER(Masks), POINTER(Tensor)]),
            "sqc_contract_workspace_bytes": (c_size_t, [POINTER(Tensor), c_int32, POINTER(Cut),
                                                        c_int32, c_int]),
            "sqc_contract": (c_int, [P, POINTER(Tensor), c_int32, POINTER(Cut), c_int32, c_int,
                                     P, c_int]),
            "sqc_contract_sliced_workspace_bytes": (c_size_t, [POINTER(Tensor), c_int32,
                                                               POINTER(Cut), c_int32,
                                                               POINTER(c_int32), c_int32, c_int]),
            "sqc_contract_sliced": (c_int, [P, POINTER(Tensor), c_int32, POINTER(Cut), c_int32,
                                            POINTER(c_int32), c_int32, c_int, P, c_int]),
            "sqc_query_states_workspace_bytes": (c_size_t, [POINTER(Tensor), c_int32, POINTER(Cut),
                                                            c_int32, c_int]),
            "sqc_query_states": (c_int, [P, POINTER(Tensor), c_int32, POINTER(Cut), c_int32,
                                         POINTER(c_uint64), ctypes.c_int64, c_int, P, c_int]),
            "sqc_recurse_workspace_bytes": (c_size_t, [POINTER(Tensor), c_int32, POINTER(Cut),
                                                       c_int32, POINTER(Masks), c_int]),
            "sqc_recurse_slices": (c_int, [POINTER(Tensor), c_int32, POINTER(Cut), c_int32,
                                           POINTER(Masks), c_int, c_int32, c_size_t, POINTER(c_int32),
                                           POINTER(c_int32), POINTER(c_size_t)]),
            "sqc_recurse": (c_int, [P, POINTER(Tensor), c_int32, POINTER(Cut), c_int32,
                                    POINTER(Masks), c_uint64, c_int32, c_int, P, c_int,
                                    POINTER(Masks), P, P]),
            "sqc_recurse_noalloc": (c_int, [P, POINTER(Tensor), c_int32, POINTER(Cut), c_int32,
                                            POINTER(Masks), c_uint64, c_int32, c_int, P, c_int,
                                            POINTER(Masks), P, P]),
            "sqc_ctx_set_tolerance": (c_int, [P, c_double]),
            "sqc_select_precision": (c_int, [P, POINTER(Tensor), c_int32, POINTER(Cut), c_int32, POINTER(Masks),
                                             c_uint64, POINTER(c_int), POINTER(c_double)]),
            "sqc_ctx_auto_choice": (c_int, [P, POINTER(c_int), POINTER(c_double)]),
            "sqc_search_workspace_bytes": (c_size_t, [POINTER(Tensor), c_int32, POINTER(Cut), c_int32,
                                                      c_uint64, c_int32, c_int, c_int32]),
            "sqc_search": (c_int, [P, POINTER(Tensor), c_int32, POINTER(Cut), c_int32, c_uint64,
                                   c_int32, c_int, P, c_int, POINTER(Found), POINTER(c_uint64),
                                   c_int32, POINTER(c_int32), POINTER(RecursionInfo),
                                   POINTER(c_int32)]),
            "sqc_autotune": (c_int, [P, POINTER(Tensor), c_int32, POINTER(Cut), c_int32, POINTER(Masks),
                                     c_uint64, c_int, P, c_int, c_int32, POINTER(TuneReport)]),
            "sqc_autotune_reset": (c_int, []),
            "sqc_graph_begin": (c_int, [P]),
            "sqc_graph_end": (c_int, [P, POINTER(P)]),
            "sqc_graph_launch": (c_int, [P, P]),
            "sqc_graph_destroy": (c_int, [P]),
            "sqc_autotune_entries": (c_int32, []),
            "sqc_serve_create": (c_int, [c_int, c_int32, P, c_size_t, POINTER(P)]),
            "sqc_serve_destroy": (c_int, [P]),
            "sqc_serve_set_max_batch": (c_int, [P, c_int32]),
            "sqc_serve_register": (c_int, [P, POINTER(Tensor), c_int32, POINTER(Cut), c_int32,
                                           POINTER(c_int32)]),
            "sqc_serve_footprint": (c_size_t, [P, POINTER(Request)]),
            "sqc_serve_submit": (c_int, [P, POINTER(Request), POINTER(c_uint64)]),
            "sqc_serve_submit_many": (c_int, [P, POINTER(Request), c_int32, POINTER(c_uint64)]),
            "sqc_serve_poll": (c_int, [P, c_uint64, POINTER(c_int32)]),
            "sqc_serve_wait": (c_int, [P, c_uint64]),
            "sqc_serve_get_stats": (c_int, [P, POINTER(ServeStats)]),
            "sqc_serve_pick_batch": (c_int, [POINTER(c_size_t), POINTER(c_size_t), POINTER(c_int32), c_int32,
                                             c_size_t, c_int32, POINTER(c_int32), POINTER(c_int32),
                                             POINTER(c_int32)]),
            "sqc_serve_completed": (c_int, [P, POINTER(c_uint64), c_int32, POINTER(c_int32)]),
            "sqc_serve_last_error": (c_char_p, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _typed.update(sig)
        _lib = L
    return _lib


_typed = set()  # entry points given a ctypes signature by lib()


def typed_symbols() -> List[str]:
    """Entry points the binding declares argument and result types for."""
    lib()
    return sorted(_typed)


def declared_symbols() -> List[str]:
    """Names of the functions the public header declares."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "sqc.h")
    txt = open(hdr).read()
    return sorted(set(re.findall(r"\b(sqc_[a-z_]+)\s*\(", txt)))


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

class Graph:
    """C arrays describing a compute graph (keeps the data_wire arrays alive)."""

    def __init__(self, n_wires: Sequence[int], data_wire: Sequence[Sequence[int]],
                 cuts: Sequence[Sequence[int]]):
        self.n_sub = len(n_wires)
        self._dw = [(c_int32 * max(1, len(dw)))(*dw) for dw in data_wire]
        self.subs = (Sub * self.n_sub)()
        for i in range(self.n_sub):
            self.subs[i].n_wires = int(n_wires[i])
            self.subs[i].n_data = len(data_wire[i])
            self.subs[i].data_wire = ctypes.cast(self._dw[i], POINTER(c_int32))
        self.n_cuts = len(cuts)
        self.cuts = (Cut * max(1, self.n_cuts))()
        for k, c in enumerate(cuts):
            self.cuts[k].up_sub, self.cuts[k].up_wire, self.cuts[k].down_sub, self.cuts[k].down_wire = (
                int(c[0]), int(c[1]), int(c[2]), int(c[3]))
        self.n_data = [len(dw) for dw in data_wire]
        self.degree = [sum(1 for c in cuts if c[0] == i or c[2] == i) for i in range(self.n_sub)]

    @classmethod
    def from_cut_circuit(cls, cc) -> "Graph":
        return cls([s.n_wires for s in cc.subs], [list(s.data_wire) for s in cc.subs],
                   [(c.up_sub, c.up_wire, c.down_sub, c.down_wire) for c in cc.cuts])


def _check(status: int, ctx=None):
    if status != OK:
        msg = lib().sqc_last_error(ctx).decode()
        raise SqcError(status, msg)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def masks_array(ms) -> "ctypes.Array":
    arr = (Masks * len(ms))()
    for i, m in enumerate(ms):
        if isinstance(m, Masks):
            arr[i] = m
        else:
            arr[i].fixed, arr[i].fixed_val, arr[i].active, arr[i].merged = (int(v) for v in m)
    return arr


def tensor_desc(t, n_labels: int, n_bits: int, prec: int, layout: int) -> Tensor:
    d = Tensor()
    d.data = _ptr(t)
    d.n_labels, d.n_bits, d.prec, d.layout = n_labels, n_bits, prec, layout
    return d


def tensor_array(descs: Sequence[Tensor]) -> "ctypes.Array":
    arr = (Tensor * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = d
    return arr


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def version() -> str:
    return lib().sqc_version().decode()


def ctx_create(device: int = 0, stream: Optional[int] = None) -> int:
    h = c_void_p()
    _check(lib().sqc_ctx_create(device, stream, ctypes.byref(h)))
    return h.value


def ctx_destroy(ctx: int) -> None:
    _check(lib().sqc_ctx_destroy(ctx), None)


def ctx_set_stream(ctx: int, stream: Optional[int]) -> None:
    _check(lib().sqc_ctx_set_stream(ctx, stream), ctx)


def ctx_set_workspace(ctx: int, buf) -> None:
    _check(lib().sqc_ctx_set_workspace(ctx, _ptr(buf), buf.numel() * buf.element_size()), ctx)


def ctx_set_timing(ctx: int, mask: int) -> None:
    _check(lib().sqc_ctx_set_timing(ctx, mask), ctx)


def ctx_timing(ctx: int, stage: int, reset: bool = False) -> StageTime:
    out = StageTime()
    _check(lib().sqc_ctx_timing(ctx, stage, 1 if reset else 0, ctypes.byref(out)), ctx)
    return out


def check_graph(g: Graph) -> None:
    _check(lib().sqc_check_graph(g.subs, g.n_sub, g.cuts, g.n_cuts))


def assign_bins(n_data: Sequence[int], scope, M: int) -> List[Masks]:
    n = len(n_data)
    nd = (c_int32 * n)(*n_data)
    sc = masks_array(scope) if scope is not None else None
    out = (Masks * n)()
    _check(lib().sqc_assign_bins(n, nd, sc, M, out))
    return list(out)


def bin_scope(masks, b: int) -> List[Masks]:
    arr = masks_array(masks)
    out = (Masks * len(arr))()
    _check(lib().sqc_bin_scope(len(arr), arr, b, out))
    return list(out)


def plan_cost(out_bits: Sequence[int], cuts: Sequence[Sequence[int]],
              order: Optional[Sequence[int]] = None) -> Cost:
    n = len(out_bits)
    ob = (c_int32 * n)(*out_bits)
    cs = (Cut * max(1, len(cuts)))()
    for k, c in enumerate(cuts):
        cs[k].up_sub, cs[k].down_sub = int(c[0]), int(c[1])
    od = (c_int32 * len(order))(*order) if order is not None else None
    out = Cost()
    _check(lib().sqc_plan_cost(n, ob, cs, len(cuts), od, ctypes.byref(out)))
    return out


def slice_plan(out_bits: Sequence[int], cuts: Sequence[Sequence[int]], budget: float) -> List[int]:
    n = len(out_bits)
    ob = (c_int32 * n)(*out_bits)
    cs = (Cut * max(1, len(cuts)))()
    for k, c in enumerate(cuts):
        cs[k].up_sub, cs[k].down_sub = int(c[0]), int(c[1])
    sl = (c_int32 * max(1, len(cuts)))()
    ns = c_int32()
    _check(lib().sqc_slice_plan(n, ob, cs, len(cuts), float(budget), sl, ctypes.byref(ns)))
    return list(sl[:ns.value])


def find_cuts(n_qubits: int, gates: Sequence[Sequence[int]], n_sub: int, alpha: float,
              max_nodes: int = 0):
    """Cut search of Sec. 5: (assignment per gate, L, cut edges, optimal)."""
    n = len(gates)
    flat = (c_int32 * max(2, 2 * n))(*[int(q) for g in gates for q in g])
    out = (c_int32 * max(1, n))()
    L, nc, opt = c_int32(), c_int32(), c_int32()
    _check(lib().sqc_find_cuts(n_qubits, flat, n, n_sub, float(alpha), int(max_nodes), out,
                               ctypes.byref(L), ctypes.byref(nc), ctypes.byref(opt)))
    return list(out[:n]), L.value, nc.value, bool(opt.value)


def attribute_bytes(g: Graph, sub_id: int, out_prec: int) -> int:
    return int(lib().sqc_attribute_bytes(g.subs, g.n_sub, sub_id, g.cuts, g.n_cuts, out_prec))


def attribute(ctx: int, g: Graph, sub_id: int, variants, in_prec: int, out, out_prec: int) -> Tensor:
    d = Tensor()
    d.data = _ptr(out)
    d.prec = out_prec
    _check(lib().sqc_attribute(ctx, g.subs, g.n_sub, sub_id, g.cuts, g.n_cuts, _ptr(variants),
                               in_prec, ctypes.byref(d)), ctx)
    return d


def attribute_all(ctx: int, g: Graph, variants, in_prec: int, outs, out_prec: int) -> List[Tensor]:
    n = g.n_sub
    vp = (c_void_p * n)(*[_ptr(v) for v in variants])
    arr = (Tensor * n)()
    for i in range(n):
        arr[i].data = _ptr(outs[i])
        arr[i].prec = out_prec
    _check(lib().sqc_attribute_all(ctx, g.subs, n, g.cuts, g.n_cuts, vp, in_prec, arr), ctx)
    return list(arr)


def attribute_all_merged(ctx: int, g: Graph, variants, in_prec: int, outs, out_prec: int) -> List[Tensor]:
    """sqc_attribute_all_merged: every subcircuit attributed straight into
    the merged layout of a recursion that keeps all its data bits active."""
    n = g.n_sub
    vp = (c_void_p * n)(*[_ptr(v) for v in variants])
    arr = (Tensor * n)()
    for i in range(n):
        arr[i].data = _ptr(outs[i])
        arr[i].prec = out_prec
    _check(lib().sqc_attribute_all_merged(ctx, g.subs, n, g.cuts, g.n_cuts, vp, in_prec, arr), ctx)
    return list(arr)


def merge_workspace_bytes(att: Tensor, masks) -> int:
    m = masks_array([masks])
    return int(lib().sqc_merge_workspace_bytes(ctypes.byref(att), m))


def merge(ctx: int, att: Tensor, masks, out, out_prec: int) -> Tensor:
    m = masks_array([masks])
    d = Tensor()
    d.data = _ptr(out)
    d.prec = out_prec
    _check(lib().sqc_merge(ctx, ctypes.byref(att), m, ctypes.byref(d)), ctx)
    return d


def contract_workspace_bytes(merged: Sequence[Tensor], g: Graph, prec: int) -> int:
    arr = tensor_array(merged)
    return int(lib().sqc_contract_workspace_bytes(arr, g.n_sub, g.cuts, g.n_cuts, prec))


def contract(ctx: int, merged: Sequence[Tensor], g: Graph, prec: int, bins, bins_prec: int) -> None:
    arr = tensor_array(merged)
    _check(lib().sqc_contract(ctx, arr, g.n_sub, g.cuts, g.n_cuts, prec, _ptr(bins), bins_prec), ctx)


def _sliced_array(sliced: Sequence[int]):
    return (c_int32 * max(1, len(sliced)))(*[int(k) for k in sliced])


def contract_sliced_workspace_bytes(merged: Sequence[Tensor], g: Graph, sliced: Sequence[int],
                                    prec: int) -> int:
    arr = tensor_array(merged)
    return int(lib().sqc_contract_sliced_workspace_bytes(arr, g.n_sub, g.cuts, g.n_cuts,
                                                         _sliced_array(sliced), len(sliced), prec))


def contract_sliced(ctx: int, merged: Sequence[Tensor], g: Graph, sliced: Sequence[int], prec: int,
                    bins, bins_prec: int) -> None:
    arr = tensor_array(merged)
    _check(lib().sqc_contract_sliced(ctx, arr, g.n_sub, g.cuts, g.n_cuts, _sliced_array(sliced),
                                     len(sliced), prec, _ptr(bins), bins_prec), ctx)


def query_states_workspace_bytes(att: Sequence[Tensor], g: Graph, prec: int) -> int:
    arr = tensor_array(att)
    return int(lib().sqc_query_states_workspace_bytes(arr, g.n_sub, g.cuts, g.n_cuts, prec))


def query_states(ctx: int, att: Sequence[Tensor], g: Graph, states: Sequence[int], prec: int, probs,
                 probs_prec: int) -> None:
    arr = tensor_array(att)
    st = (c_uint64 * max(1, len(states)))(*[int(x) for x in states])
    _check(lib().sqc_query_states(ctx, arr, g.n_sub, g.cuts, g.n_cuts, st, len(states), prec, _ptr(probs),
                                  probs_prec), ctx)


def recurse_workspace_bytes(att: Sequence[Tensor], g: Graph, masks, prec: int) -> int:
    arr = tensor_array(att)
    m = masks_array(masks)
    return int(lib().sqc_recurse_workspace_bytes(arr, g.n_sub, g.cuts, g.n_cuts, m, prec))


def recurse_slices(att: Sequence[Tensor], g: Graph, masks, prec: int, top_r: int,
                   workspace_bytes: int):
    """Cuts sqc_recurse slices under a workspace of that size (Sec. 6.3):
    (cut ids in slice-digit order, bytes the chosen layout needs)."""
    arr = tensor_array(att)
    m = masks_array(masks)
    sl = (c_int32 * MAX_SLICED)()
    ns = c_int32()
    need = c_size_t()
    _check(lib().sqc_recurse_slices(arr, g.n_sub, g.cuts, g.n_cuts, m, prec, top_r, int(workspace_bytes), sl,
                                    ctypes.byref(ns), ctypes.byref(need)))
    return list(sl[:ns.value]), int(need.value)


def recurse(ctx: int, att: Sequence[Tensor], g: Graph, scope, M: int, top_r: int, prec: int,
            bins, bins_prec: int, topr, bsum) -> List[Masks]:
    arr = tensor_array(att)
    sc = masks_array(scope) if scope is not None else None
    out = (Masks * g.n_sub)()
    _check(lib().sqc_recurse(ctx, arr, g.n_sub, g.cuts, g.n_cuts, sc, M, top_r, prec, _ptr(bins),
                             bins_prec, out, _ptr(topr), _ptr(bsum)), ctx)
    return list(out)


def recurse_noalloc(ctx: int, att: Sequence[Tensor], g: Graph, scope, M: int, top_r: int, prec: int,
                    bins, bins_prec: int, topr, bsum) -> List[Masks]:
    arr = tensor_array(att)
    sc = masks_array(scope) if scope is not None else None
    out = (Masks * g.n_sub)()
    _check(lib().sqc_recurse_noalloc(ctx, arr, g.n_sub, g.cuts, g.n_cuts, sc, M, top_r, prec, _ptr(bins),
                                     bins_prec, out, _ptr(topr), _ptr(bsum)), ctx)
    return list(out)


def autotune(ctx: int, att: Sequence[Tensor], g: Graph, scope, M: int, prec: int, bins,
             bins_prec: int, reps: int = 5) -> TuneReport:
    arr = tensor_array(att)
    sc = masks_array(scope) if scope is not None else None
    rep = TuneReport()
    _check(lib().sqc_autotune(ctx, arr, g.n_sub, g.cuts, g.n_cuts, sc, M, prec, _ptr(bins), bins_prec,
                              reps, ctypes.byref(rep)), ctx)
    return rep


def graph_begin(ctx: int) -> None:
    _check(lib().sqc_graph_begin(ctx), ctx)


def graph_end(ctx: int) -> int:
    h = c_void_p()
    _check(lib().sqc_graph_end(ctx, ctypes.byref(h)), ctx)
    return h.value


def graph_launch(ctx: int, graph: int) -> None:
    _check(lib().sqc_graph_launch(ctx, graph), ctx)


def graph_destroy(graph: int) -> None:
    _check(lib().sqc_graph_destroy(graph))


def autotune_reset() -> None:
    _check(lib().sqc_autotune_reset())


def autotune_entries() -> int:
    return int(lib().sqc_autotune_entries())


def ctx_set_tolerance(ctx: int, max_abs_error: float) -> None:
    _check(lib().sqc_ctx_set_tolerance(ctx, max_abs_error), ctx)


def select_precision(ctx: int, att: Sequence[Tensor], g: Graph, scope, M: int):
    """(chosen precision, certified bound of the bins' sums of |terms|)."""
    arr = tensor_array(att)
    sc = masks_array(scope) if scope is not None else None
    ch, b = c_int(), c_double()
    _check(lib().sqc_select_precision(ctx, arr, g.n_sub, g.cuts, g.n_cuts, sc, M, ctypes.byref(ch),
                                      ctypes.byref(b)), ctx)
    return ch.value, b.value


def ctx_auto_choice(ctx: int):
    ch, b = c_int(), c_double()
    _check(lib().sqc_ctx_auto_choice(ctx, ctypes.byref(ch), ctypes.byref(b)), ctx)
    return ch.value, b.value


def search_workspace_bytes(att: Sequence[Tensor], g: Graph, M: int, R: int, prec: int,
                           max_solutions: int = 64) -> int:
    arr = tensor_array(att)
    return int(lib().sqc_search_workspace_bytes(arr, g.n_sub, g.cuts, g.n_cuts, M, R, prec, max_solutions))


def search(ctx: int, att: Sequence[Tensor], g: Graph, M: int, R: int, prec: int, bins,
           bins_prec: int, max_solutions: int = 64):
    arr = tensor_array(att)
    sol = (Found * max(1, max_solutions))()
    states = (c_uint64 * max(1, max_solutions * g.n_sub))()
    nsol = c_int32()
    info = (RecursionInfo * R)()
    nrec = c_int32()
    _check(lib().sqc_search(ctx, arr, g.n_sub, g.cuts, g.n_cuts, M, R, prec, _ptr(bins), bins_prec,
                            sol, states, max_solutions, ctypes.byref(nsol), info,
                            ctypes.byref(nrec)), ctx)
    sols = []
    for k in range(nsol.value):
        sols.append((sol[k].prob, sol[k].recursion, sol[k].bin,
                     [states[k * g.n_sub + i] for i in range(g.n_sub)]))
    infos = [(info[r].bins_sum, info[r].parent_prob, info[r].top_prob, info[r].active_bits,
              bool(info[r].leaf)) for r in range(nrec.value)]
    return sols, infos


# ---------------------------------------------------------------------------
# serving engine
# ---------------------------------------------------------------------------

def _check_srv(status: int, srv):
    if status != OK:
        raise SqcError(status, lib().sqc_serve_last_error(srv).decode())


def serve_create(device: int, n_slots: int, workspace) -> int:
    h = c_void_p()
    _check(lib().sqc_serve_create(device, n_slots, _ptr(workspace),
                                  workspace.numel() * workspace.element_size(), ctypes.byref(h)))
    return h.value


def serve_set_max_batch(srv: int, max_batch: int) -> None:
    _check_srv(lib().sqc_serve_set_max_batch(srv, max_batch), srv)


def serve_destroy(srv: int) -> None:
    _check(lib().sqc_serve_destroy(srv))


def serve_register(srv: int, att: Sequence[Tensor], g: Graph) -> int:
    cid = c_int32()
    _check_srv(lib().sqc_serve_register(srv, tensor_array(att), g.n_sub, g.cuts, g.n_cuts,
                                        ctypes.byref(cid)), srv)
    return cid.value


def make_request(circuit: int, n_sub: int, scope, M: int, top_r: int, prec: int, bins,
                 bins_prec: int, topr, bsum, masks_out=None) -> Request:
    """A request struct; the scope and masks arrays it points to are kept on
    the struct (``_keep``) so they outlive the call."""
    r = Request()
    r.circuit, r.top_r, r.max_bins_M, r.prec, r.bins_prec = circuit, top_r, M, prec, bins_prec
    keep = []
    if scope is not None:
        sc = masks_array(scope)
        keep.append(sc)
        r.scope = ctypes.cast(sc, POINTER(Masks))
    if masks_out is not None:
        keep.append(masks_out)
        r.masks_out = ctypes.cast(masks_out, POINTER(Masks))
    r.bins_dev, r.topr_dev, r.sum_dev = _ptr(bins), _ptr(topr), _ptr(bsum)
    r._keep = keep
    return r


def serve_footprint(srv: int, req: Request) -> int:
    return int(lib().sqc_serve_footprint(srv, ctypes.byref(req)))


def serve_submit(srv: int, req: Request) -> int:
    t = c_uint64()
    _check_srv(lib().sqc_serve_submit(srv, ctypes.byref(req), ctypes.byref(t)), srv)
    return t.value


def serve_submit_many(srv: int, reqs: Sequence[Request]) -> List[int]:
    n = len(reqs)
    arr = (Request * max(1, n))()
    for k, r in enumerate(reqs):
        arr[k] = r  # (a copy: the scope and masks_out pointers stay the caller's)
    out = (c_uint64 * max(1, n))()
    _check_srv(lib().sqc_serve_submit_many(srv, arr, n, out), srv)
    return list(out[:n])


def serve_poll(srv: int, ticket: int) -> int:
    st = c_int32()
    _check_srv(lib().sqc_serve_poll(srv, ticket, ctypes.byref(st)), srv)
    return st.value


def serve_wait(srv: int, ticket: int) -> None:
    _check_srv(lib().sqc_serve_wait(srv, ticket), srv)


def serve_completed(srv: int, cap: int = 256) -> List[int]:
    buf = (c_uint64 * max(1, cap))()
    n = c_int32()
    _check_srv(lib().sqc_serve_completed(srv, buf, cap, ctypes.byref(n)), srv)
    return [buf[k] for k in range(n.value)]


def serve_pick_batch(ws_bytes: Sequence[int], table_bytes: Sequence[int], skips: List[int], room: int,
                     max_batch: int):
    """The serving engine's batching policy: (positions taken, held by an
    aged request); `skips` is updated in place."""
    n = len(ws_bytes)
    w = (c_size_t * max(1, n))(*ws_bytes)
    t = (c_size_t * max(1, n))(*table_bytes)
    sk = (c_int32 * max(1, n))(*skips)
    out = (c_int32 * max(1, n))()
    npk, held = c_int32(), c_int32()
    st = lib().sqc_serve_pick_batch(w, t, sk, n, int(room), int(max_batch), out, ctypes.byref(npk),
                                    ctypes.byref(held))
    if st != OK:
        raise SqcError(st, "sqc_serve_pick_batch: invalid argument")
    skips[:] = list(sk[:n])
    return list(out[:npk.value]), bool(held.value)


def serve_get_stats(srv: int) -> ServeStats:
    out = ServeStats()
    _check(lib().sqc_serve_get_stats(srv, ctypes.byref(out)))
    return out
