"""Python binding of the MI355X probe library (libgace.so, C ABI in include/gace.h).

Argument marshalling only: every step of the probe runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and streams.  There is no
fallback: if libgace.so is missing, importing the binding's functions raises.

Names follow the C ABI: gace_create, gace_probe_selectivity, gace_join_freq,
gace_batch_run, gace_autotune, gace_server_create / submit / wait / destroy ...
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgace.so")

GACE_OK, GACE_EINVAL, GACE_ENOMEM, GACE_EOVERFLOW, GACE_EDEVICE, GACE_EBUSY, GACE_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EOVERFLOW", -4: "EDEVICE", -5: "EBUSY", -6: "ETIMEOUT"}
I32, I64, F32 = 1, 2, 3
RANGE, EQ, IN = 1, 2, 3
REQ_SELECTIVITY, REQ_JOIN = 1, 2


class GaceError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


# ---------------------------------------------------------------- C structs
class gace_column(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class gace_table(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_uint64), ("cols", ctypes.POINTER(gace_column)),
                ("n_cols", ctypes.c_uint32), ("table_id", ctypes.c_uint32)]


class gace_term(ctypes.Structure):
    _fields_ = [("col", ctypes.c_uint32), ("op", ctypes.c_uint32), ("n_vals", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("v", ctypes.c_int64 * 8)]


class gace_predicates(ctypes.Structure):
    _fields_ = [("terms", ctypes.POINTER(gace_term)), ("pred_off", ctypes.POINTER(ctypes.c_uint32)),
                ("n_preds", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class gace_sample_spec(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("rate", ctypes.c_double), ("block_rows", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class gace_probe_info(ctypes.Structure):
    _fields_ = [("sampled_rows", ctypes.c_uint64), ("kept_blocks", ctypes.c_uint64)]


class gace_keys(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("n", ctypes.c_uint64), ("table_id", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("spec", gace_sample_spec)]


JOIN_FIELDS = ("join_card", "ndv_R", "ndv_S", "n_R", "n_S", "f1_R", "f1_S", "f2_R", "f2_S")


class gace_join_result(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in JOIN_FIELDS]


def _join_dict(o) -> dict:
    return {n: int(getattr(o, n)) for n in JOIN_FIELDS}


class gace_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("table", gace_table), ("preds", gace_predicates), ("spec", gace_sample_spec),
                ("counts", ctypes.POINTER(ctypes.c_uint64)), ("info", ctypes.POINTER(gace_probe_info)),
                ("R", gace_keys), ("S", gace_keys), ("join", ctypes.POINTER(gace_join_result))]


class gace_schedule(ctypes.Structure):
    _fields_ = [("wg_threads", ctypes.c_uint32), ("wgs_per_cu", ctypes.c_uint32), ("item_rows", ctypes.c_uint32),
                ("count_mode", ctypes.c_uint32), ("join_part_keys", ctypes.c_uint32),
                ("join_wgs_per_cu", ctypes.c_uint32), ("agg_wgs_per_cu", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class gace_trace_rec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("index", ctypes.c_uint32), ("wg", ctypes.c_uint32),
                ("xcc", ctypes.c_uint32), ("t_begin", ctypes.c_uint64), ("t_ready", ctypes.c_uint64),
                ("t_end", ctypes.c_uint64), ("work", ctypes.c_uint64)]


class gace_kernel_stats(ctypes.Structure):
    _fields_ = [("scan_ms", ctypes.c_double), ("join_ms", ctypes.c_double), ("scan_alg_bytes", ctypes.c_uint64),
                ("join_alg_bytes", ctypes.c_uint64), ("timed", ctypes.c_uint32), ("compile_ms", ctypes.c_float),
                ("zones_skipped", ctypes.c_uint64)]


class gace_server_cfg(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("queue_capacity", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("workspace_bytes", ctypes.c_uint64)]


class gace_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "rejected", "batches", "queued",
                                                "inflight", "workspace_in_use", "workspace_peak",
                                                "completed_early")]


# gace_gate.h
GATE_DRIFT, GATE_SELERR, GATE_PCS, GATE_PCS_HI, GATE_PCS_LO = 1, 2, 4, 4, 8


class gace_gate_cfg(ctypes.Structure):
    _fields_ = [("drift_min", ctypes.c_double), ("sel_err_max", ctypes.c_double),
                ("pcs_hi_num", ctypes.c_uint32), ("pcs_hi_den", ctypes.c_uint32),
                ("pcs_lo_num", ctypes.c_uint32), ("pcs_lo_den", ctypes.c_uint32)]


class gace_gate_in(ctypes.Structure):
    _fields_ = [("have", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("ndv_hist", ctypes.c_double),
                ("ndv_est", ctypes.c_double), ("s_est", ctypes.c_double), ("count", ctypes.c_uint64),
                ("n", ctypes.c_uint64), ("c_ab", ctypes.c_uint64), ("c_a", ctypes.c_uint64),
                ("c_b", ctypes.c_uint64), ("n_pcs", ctypes.c_uint64)]


class gace_gate_out(ctypes.Structure):
    _fields_ = [("drift", ctypes.c_double), ("sel_err", ctypes.c_double), ("pcs", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("undefined", ctypes.c_uint32), ("trigger", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class gace_cost_features(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_double), ("row_bytes", ctypes.c_double), ("terms", ctypes.c_double),
                ("reserved", ctypes.c_double)]


class gace_cache_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("hits", "misses", "inserts", "evictions", "invalidated", "entries")]


# gace_host.h
class gace_host_opts(ctypes.Structure):
    _fields_ = [("key_only", ctypes.c_uint32), ("gather_threads", ctypes.c_uint32), ("chunk_rows", ctypes.c_uint64)]


class gace_transfer_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("total_ms", "sample_ms", "gather_ms", "h2d_ms", "kernel_ms",
                                               "d2h_ms", "reduce_ms")] + \
               [("h2d_bytes", ctypes.c_uint64), ("chunks", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


# gace_est.h
class gace_sel_estimate(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("p", "sel", "card", "card_ht")]


class gace_join_estimate(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("p_R", "p_S", "join_ht", "ndv_R", "ndv_S")]


ABI_FUNCTIONS = [
    "gace_create", "gace_destroy", "gace_last_error", "gace_version", "gace_check_request",
    "gace_probe_selectivity", "gace_join_freq", "gace_batch_run", "gace_autotune", "gace_get_schedule",
    "gace_set_schedule", "gace_last_batch_stats", "gace_last_kernel_stats", "gace_set_graph",
    "gace_set_trace", "gace_get_trace", "gace_set_spin_limit",
    "gace_server_create", "gace_server_submit",
    "gace_server_wait", "gace_server_wait_times", "gace_server_stats_get", "gace_server_destroy",
    # gace_gate.h
    "gace_gate_default_cfg", "gace_gate_evaluate", "gace_probe_pcs",
    "gace_cost_create", "gace_cost_destroy", "gace_cost_observe", "gace_cost_coef", "gace_cost_predict",
    "gace_cost_features_of", "gace_cost_breakeven",
    "gace_cache_create", "gace_cache_destroy", "gace_cache_lookup", "gace_cache_insert", "gace_cache_invalidate",
    "gace_cache_stats_get", "gace_probe_selectivity_cached", "gace_join_freq_cached",
    # gace_host.h
    "gace_probe_selectivity_host",
    # gace_est.h
    "gace_estimate_selectivity", "gace_estimate_join",
    # gace_zone.h
    "gace_zonemap_build", "gace_zonemap_destroy", "gace_zonemap_info", "gace_zonemap_read",
    "gace_probe_selectivity_zm", "gace_zonemap_attach", "gace_zonemap_detach", "gace_server_attach_zonemap",
    "gace_probe_selectivity_noalloc",
    "gace_read_ceiling",
]

_lib = None


def lib():
    """Load libgace.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except Exception:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgace.so is not built: run python paper_2512_19750_amd/build.py first")
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        sig = {
            "gace_create": ([ctypes.c_int, u64, ctypes.POINTER(P)], i32),
            "gace_destroy": ([P], i32),
            "gace_last_error": ([], ctypes.c_char_p),
            "gace_version": ([], ctypes.c_char_p),
            "gace_check_request": ([ctypes.POINTER(gace_request)], i32),
            "gace_probe_selectivity": ([P, ctypes.POINTER(gace_table), ctypes.POINTER(gace_predicates),
                                        ctypes.POINTER(gace_sample_spec), ctypes.POINTER(ctypes.c_uint64),
                                        ctypes.POINTER(gace_probe_info), P], i32),
            "gace_read_ceiling": ([P, u64, P, ctypes.POINTER(ctypes.c_double), P], i32),
            "gace_probe_selectivity_noalloc": ([ctypes.POINTER(gace_table), ctypes.POINTER(gace_predicates),
                                                ctypes.POINTER(gace_sample_spec), ctypes.POINTER(ctypes.c_uint64),
                                                ctypes.POINTER(gace_probe_info), P], i32),
            "gace_join_freq": ([P, ctypes.POINTER(gace_keys), ctypes.POINTER(gace_keys),
                                ctypes.POINTER(gace_join_result), P], i32),
            "gace_batch_run": ([P, ctypes.POINTER(gace_request), u32, ctypes.POINTER(i32), P], i32),
            "gace_autotune": ([P, ctypes.POINTER(gace_request), u32, ctypes.c_char_p, P], i32),
            "gace_get_schedule": ([P, ctypes.POINTER(gace_schedule)], i32),
            "gace_set_schedule": ([P, ctypes.POINTER(gace_schedule)], i32),
            "gace_last_batch_stats": ([P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64),
                                       ctypes.POINTER(u64)], i32),
            "gace_last_kernel_stats": ([P, ctypes.POINTER(gace_kernel_stats)], i32),
            "gace_set_graph": ([P, ctypes.c_int], i32),
            "gace_set_trace": ([P, ctypes.c_int], i32),
            "gace_set_spin_limit": ([P, u64], i32),
            "gace_get_trace": ([P, ctypes.POINTER(gace_trace_rec), u32, ctypes.POINTER(u32),
                                ctypes.POINTER(ctypes.c_double)], i32),
            "gace_server_create": ([ctypes.c_int, ctypes.POINTER(gace_server_cfg), ctypes.POINTER(P)], i32),
            "gace_server_submit": ([P, ctypes.POINTER(gace_request), ctypes.POINTER(u64)], i32),
            "gace_server_wait": ([P, u64, ctypes.c_int64, ctypes.POINTER(i32)], i32),
            "gace_server_wait_times": ([P, u64, ctypes.c_int64, ctypes.POINTER(i32), ctypes.POINTER(u64),
                                        ctypes.POINTER(u64)], i32),
            "gace_server_stats_get": ([P, ctypes.POINTER(gace_server_stats)], i32),
            "gace_server_destroy": ([P], i32),
            "gace_gate_default_cfg": ([ctypes.POINTER(gace_gate_cfg)], i32),
            "gace_gate_evaluate": ([ctypes.POINTER(gace_gate_cfg), ctypes.POINTER(gace_gate_in),
                                    ctypes.POINTER(gace_gate_out)], i32),
            "gace_probe_pcs": ([P, ctypes.POINTER(gace_table), ctypes.POINTER(gace_predicates),
                                ctypes.POINTER(gace_sample_spec), ctypes.POINTER(gace_gate_in), P], i32),
            "gace_cost_create": ([ctypes.c_double, u32, ctypes.POINTER(P)], i32),
            "gace_cost_destroy": ([P], i32),
            "gace_cost_observe": ([P, ctypes.POINTER(gace_cost_features), ctypes.c_double], i32),
            "gace_cost_coef": ([P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u32)], i32),
            "gace_cost_predict": ([P, ctypes.POINTER(gace_cost_features), ctypes.POINTER(ctypes.c_double)], i32),
            "gace_cost_features_of": ([ctypes.POINTER(gace_request), ctypes.POINTER(gace_cost_features)], i32),
            "gace_cost_breakeven": ([P, P, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double)],
                                    i32),
            "gace_cache_create": ([u64, ctypes.POINTER(P)], i32),
            "gace_cache_destroy": ([P], i32),
            "gace_cache_lookup": ([P, ctypes.POINTER(gace_table), ctypes.POINTER(gace_predicates),
                                   ctypes.POINTER(gace_sample_spec), ctypes.POINTER(u64),
                                   ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(gace_probe_info),
                                   ctypes.POINTER(u32)], i32),
            "gace_cache_insert": ([P, ctypes.POINTER(gace_table), ctypes.POINTER(gace_predicates),
                                   ctypes.POINTER(gace_sample_spec), ctypes.POINTER(u64),
                                   ctypes.POINTER(gace_probe_info)], i32),
            "gace_cache_invalidate": ([P, u32], i32),
            "gace_cache_stats_get": ([P, ctypes.POINTER(gace_cache_stats)], i32),
            "gace_probe_selectivity_cached": ([P, P, ctypes.POINTER(gace_table), ctypes.POINTER(gace_predicates),
                                               ctypes.POINTER(gace_sample_spec), ctypes.POINTER(u64),
                                               ctypes.POINTER(gace_probe_info), ctypes.POINTER(u32), P], i32),
            "gace_join_freq_cached": ([P, P, ctypes.POINTER(gace_keys), ctypes.POINTER(gace_keys),
                                       ctypes.POINTER(gace_join_result), ctypes.POINTER(u32), P], i32),
            "gace_zonemap_build": ([P, ctypes.POINTER(gace_table), ctypes.POINTER(P), P], i32),
            "gace_zonemap_destroy": ([P], i32),
            "gace_zonemap_attach": ([P, P], i32),
            "gace_zonemap_detach": ([P, P], i32),
            "gace_server_attach_zonemap": ([P, P], i32),
            "gace_zonemap_info": ([P, ctypes.POINTER(u64)], i32),
            "gace_zonemap_read": ([P, u32, P, P], i32),
            "gace_probe_selectivity_zm": ([P, ctypes.POINTER(gace_table), P, ctypes.POINTER(gace_predicates),
                                           ctypes.POINTER(gace_sample_spec), ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(gace_probe_info), ctypes.POINTER(u64), P], i32),
            "gace_estimate_selectivity": ([u64, ctypes.POINTER(gace_probe_info), u64, ctypes.POINTER(gace_sample_spec),
                                           ctypes.POINTER(gace_sel_estimate)], i32),
            "gace_estimate_join": ([ctypes.POINTER(gace_join_result), u64, ctypes.POINTER(gace_sample_spec), u64,
                                    ctypes.POINTER(gace_sample_spec), ctypes.POINTER(gace_join_estimate)], i32),
            "gace_probe_selectivity_host": ([P, ctypes.POINTER(gace_table), ctypes.POINTER(gace_predicates),
                                             ctypes.POINTER(gace_sample_spec), ctypes.POINTER(gace_host_opts),
                                             ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(gace_probe_info),
                                             ctypes.POINTER(gace_transfer_stats), P], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def last_error() -> str:
    return lib().gace_last_error().decode()


def _check(st: int):
    if st != GACE_OK:
        raise GaceError(st, last_error())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------- marshalling
_TORCH_DTYPE = None


def _dtype_code(t) -> int:
    import torch
    m = {torch.int32: I32, torch.int64: I64, torch.float32: F32}
    if t.dtype not in m:
        raise TypeError("column dtype must be int32, int64 or float32")
    return m[t.dtype]


@dataclass
class Table:
    """Device-resident column-major table: a list of 1-D tensors of equal length."""
    cols: list
    table_id: int

    @property
    def n_rows(self) -> int:
        return int(self.cols[0].shape[0]) if self.cols else 0


@dataclass
class Keys:
    keys: object          # 1-D int64 device tensor
    table_id: int
    seed: int = 0
    rate: float = 1.0
    block_rows: int = 4096


def _f32_bits(x) -> int:
    return int(np.array([x], dtype=np.float32).view(np.uint32)[0])


class _Keep:
    """Holds the ctypes arrays a request points to."""
    def __init__(self):
        self.objs = []

    def add(self, o):
        self.objs.append(o)
        return o


def _make_table(t: Table, keep: _Keep) -> gace_table:
    cols = keep.add((gace_column * max(len(t.cols), 1))())
    for i, c in enumerate(t.cols):
        cols[i].data = c.data_ptr()
        cols[i].dtype = _dtype_code(c)
    g = gace_table()
    g.n_rows = t.n_rows
    g.cols = ctypes.cast(cols, ctypes.POINTER(gace_column))
    g.n_cols = len(t.cols)
    g.table_id = t.table_id
    return g


def _make_preds(preds, dtypes: Sequence[int], keep: _Keep) -> gace_predicates:
    n_terms = sum(len(p) for p in preds)
    terms = keep.add((gace_term * max(n_terms, 1))())
    off = keep.add((ctypes.c_uint32 * (len(preds) + 1))())
    k = 0
    for i, p in enumerate(preds):
        for (col, op, vals) in p:
            terms[k].col = col
            terms[k].op = op
            terms[k].n_vals = len(vals)
            dt = dtypes[col] if 0 <= col < len(dtypes) else 0
            for j, v in enumerate(vals[:8]):      # the library rejects n_vals > 8 itself
                terms[k].v[j] = _f32_bits(v) if dt == F32 else int(v)
            k += 1
        off[i + 1] = k
    g = gace_predicates()
    g.terms = ctypes.cast(terms, ctypes.POINTER(gace_term))
    g.pred_off = ctypes.cast(off, ctypes.POINTER(ctypes.c_uint32))
    g.n_preds = len(preds)
    return g


def _make_spec(seed: int, rate: float, block_rows: int) -> gace_sample_spec:
    s = gace_sample_spec()
    s.seed = seed & (2**64 - 1)
    s.rate = rate
    s.block_rows = block_rows
    return s


def _make_keys(k: Keys) -> gace_keys:
    g = gace_keys()
    g.keys = k.keys.data_ptr() if k.keys is not None else 0
    g.n = int(k.keys.shape[0]) if k.keys is not None else 0
    g.table_id = k.table_id
    g.spec = _make_spec(k.seed, k.rate, k.block_rows)
    return g


class SelRequest:
    def __init__(self, table: Table, preds, seed: int = 0, rate: float = 1.0, block_rows: int = 4096):
        self.table, self.preds, self.seed, self.rate, self.block_rows = table, preds, seed, rate, block_rows
        self.counts = np.zeros(max(len(preds), 1), dtype=np.uint64)
        self.info = gace_probe_info()
        self.status = None

    def fill(self, r: gace_request, keep: _Keep):
        r.kind = REQ_SELECTIVITY
        r.table = _make_table(self.table, keep)
        r.preds = _make_preds(self.preds, [_dtype_code(c) for c in self.table.cols], keep)
        r.spec = _make_spec(self.seed, self.rate, self.block_rows)
        r.counts = self.counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        r.info = ctypes.pointer(self.info)
        keep.add(self.counts)

    def result(self):
        return self.counts[:len(self.preds)].copy(), int(self.info.sampled_rows), int(self.info.kept_blocks)


class JoinRequest:
    def __init__(self, R: Keys, S: Keys):
        self.R, self.S = R, S
        self.out = gace_join_result()
        self.status = None

    def fill(self, r: gace_request, keep: _Keep):
        r.kind = REQ_JOIN
        r.R = _make_keys(self.R)
        r.S = _make_keys(self.S)
        r.join = ctypes.pointer(self.out)

    def result(self):
        return _join_dict(self.out)


def make_requests(reqs) -> Tuple[ctypes.Array, _Keep]:
    keep = _Keep()
    arr = (gace_request * max(len(reqs), 1))()
    for i, q in enumerate(reqs):
        q.fill(arr[i], keep)
    return arr, keep


# ---------------------------------------------------------------- ABI wrappers
def gace_version() -> str:
    return lib().gace_version().decode()


def gace_create(device: int = 0, workspace_bytes: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().gace_create(device, workspace_bytes, ctypes.byref(h)))
    return h.value


def gace_destroy(ctx: int):
    _check(lib().gace_destroy(ctx))


def gace_check_request(req) -> int:
    arr, keep = make_requests([req])
    return int(lib().gace_check_request(arr))


def gace_probe_selectivity(ctx: int, table: Table, preds, seed: int = 0, rate: float = 1.0,
                           block_rows: int = 4096, stream=None):
    """-> (counts uint64[n_preds], sampled_rows, kept_blocks)"""
    keep = _Keep()
    t = _make_table(table, keep)
    p = _make_preds(preds, [_dtype_code(c) for c in table.cols], keep)
    s = _make_spec(seed, rate, block_rows)
    counts = np.zeros(max(len(preds), 1), dtype=np.uint64)
    info = gace_probe_info()
    _check(lib().gace_probe_selectivity(ctx, ctypes.byref(t), ctypes.byref(p), ctypes.byref(s),
                                        counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                        ctypes.byref(info), _stream_handle(stream)))
    return counts[:len(preds)], int(info.sampled_rows), int(info.kept_blocks)


class PreparedProbe:
    """One selectivity probe marshalled once (table, predicates, sampling spec,
    output arrays), so repeated calls go straight to the C ABI: the latency
    of a call is then the library's, not the binding's."""

    def __init__(self, table: Table, preds, seed: int = 0, rate: float = 1.0, block_rows: int = 4096):
        self._keep = _Keep()
        self.t = _make_table(table, self._keep)
        self.p = _make_preds(preds, [_dtype_code(c) for c in table.cols], self._keep)
        self.s = _make_spec(seed, rate, block_rows)
        self.n = len(preds)
        self.counts = np.zeros(max(self.n, 1), dtype=np.uint64)
        self.info = gace_probe_info()
        self._cptr = self.counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))

    def run(self, ctx: int, stream=None):
        """gace_probe_selectivity -> (counts, sampled_rows, kept_blocks); counts is reused by the next call"""
        _check(lib().gace_probe_selectivity(ctx, ctypes.byref(self.t), ctypes.byref(self.p), ctypes.byref(self.s),
                                            self._cptr, ctypes.byref(self.info), _stream_handle(stream)))
        return self.counts[:self.n], int(self.info.sampled_rows), int(self.info.kept_blocks)

    def run_noalloc(self, stream=None):
        """gace_probe_selectivity_noalloc, same results"""
        _check(lib().gace_probe_selectivity_noalloc(ctypes.byref(self.t), ctypes.byref(self.p), ctypes.byref(self.s),
                                                    self._cptr, ctypes.byref(self.info), _stream_handle(stream)))
        return self.counts[:self.n], int(self.info.sampled_rows), int(self.info.kept_blocks)


def gace_probe_selectivity_noalloc(table: Table, preds, seed: int = 0, rate: float = 1.0,
                                   block_rows: int = 4096, stream=None, counts=None):
    """As gace_probe_selectivity, on the current device, with the library's
    static scratch and no context.  counts: an optional uint64 host array of
    len(preds) entries to write into.  -> (counts, sampled_rows, kept_blocks)"""
    keep = _Keep()
    t = _make_table(table, keep)
    p = _make_preds(preds, [_dtype_code(c) for c in table.cols], keep)
    s = _make_spec(seed, rate, block_rows)
    if counts is None:
        counts = np.zeros(max(len(preds), 1), dtype=np.uint64)
    assert counts.dtype == np.uint64 and counts.flags.c_contiguous and len(counts) >= len(preds)
    info = gace_probe_info()
    _check(lib().gace_probe_selectivity_noalloc(ctypes.byref(t), ctypes.byref(p), ctypes.byref(s),
                                                counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                                ctypes.byref(info), _stream_handle(stream)))
    return counts[:len(preds)], int(info.sampled_rows), int(info.kept_blocks)


def gace_read_ceiling(data, sink, stream=None) -> float:
    """Device ms of one read of the whole device tensor `data` (16-byte
    aligned, a multiple of 16 bytes) by the read-ceiling kernel; sink: a
    device tensor of at least 4 bytes."""
    ms = ctypes.c_double()
    _check(lib().gace_read_ceiling(ctypes.c_void_p(data.data_ptr()), data.numel() * data.element_size(),
                                   ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ms), _stream_handle(stream)))
    return ms.value


def gace_join_freq(ctx: int, R: Keys, S: Keys, stream=None) -> dict:
    r, s = _make_keys(R), _make_keys(S)
    out = gace_join_result()
    _check(lib().gace_join_freq(ctx, ctypes.byref(r), ctypes.byref(s), ctypes.byref(out), _stream_handle(stream)))
    return _join_dict(out)


def gace_batch_run(ctx: int, reqs, stream=None, raise_on_error: bool = True, prepared=None) -> List[int]:
    """Runs SelRequest / JoinRequest objects in one batched launch; results land
    in each object (.result()).  Returns the per-request statuses."""
    arr, keep = prepared if prepared is not None else make_requests(reqs)
    per = (ctypes.c_int32 * max(len(reqs), 1))()
    st = lib().gace_batch_run(ctx, arr, len(reqs), per, _stream_handle(stream))
    for i, q in enumerate(reqs):
        q.status = int(per[i])
    if raise_on_error and st != GACE_OK:
        raise GaceError(st, last_error())
    return [int(per[i]) for i in range(len(reqs))]


def gace_autotune(ctx: int, reqs, cache_path: Optional[str] = None, stream=None):
    arr, keep = make_requests(reqs)
    _check(lib().gace_autotune(ctx, arr, len(reqs), cache_path.encode() if cache_path else None,
                               _stream_handle(stream)))


def gace_get_schedule(ctx: int) -> dict:
    s = gace_schedule()
    _check(lib().gace_get_schedule(ctx, ctypes.byref(s)))
    return dict(wg_threads=s.wg_threads, wgs_per_cu=s.wgs_per_cu, item_rows=s.item_rows,
                count_mode=s.count_mode, join_part_keys=s.join_part_keys, join_wgs_per_cu=s.join_wgs_per_cu,
                agg_wgs_per_cu=s.agg_wgs_per_cu)


def gace_set_schedule(ctx: int, **kw):
    s = gace_schedule()
    _check(lib().gace_get_schedule(ctx, ctypes.byref(s)))
    for k, v in kw.items():
        setattr(s, k, v)
    _check(lib().gace_set_schedule(ctx, ctypes.byref(s)))


def gace_last_batch_stats(ctx: int) -> dict:
    ms = ctypes.c_double()
    ab = ctypes.c_uint64()
    rp = ctypes.c_uint64()
    _check(lib().gace_last_batch_stats(ctx, ctypes.byref(ms), ctypes.byref(ab), ctypes.byref(rp)))
    return dict(kernel_ms=ms.value, alg_bytes=int(ab.value), rows_preds=int(rp.value))


def gace_last_kernel_stats(ctx: int) -> dict:
    k = gace_kernel_stats()
    _check(lib().gace_last_kernel_stats(ctx, ctypes.byref(k)))
    return dict(timed=bool(k.timed), scan_ms=k.scan_ms, join_ms=k.join_ms, scan_alg_bytes=int(k.scan_alg_bytes),
                join_alg_bytes=int(k.join_alg_bytes), compile_ms=float(k.compile_ms),
                zones_skipped=int(k.zones_skipped))


def gace_set_graph(ctx: int, enable: bool = True):
    _check(lib().gace_set_graph(ctx, 1 if enable else 0))


def gace_set_spin_limit(ctx: int, polls: int):
    _check(lib().gace_set_spin_limit(ctx, int(polls)))


def gace_set_trace(ctx: int, enable: bool = True):
    _check(lib().gace_set_trace(ctx, 1 if enable else 0))


def gace_get_trace(ctx: int):
    """-> (numpy structured array of the last batch's item records, ticks per microsecond)"""
    n = ctypes.c_uint32()
    tpu = ctypes.c_double()
    _check(lib().gace_get_trace(ctx, None, 0, ctypes.byref(n), ctypes.byref(tpu)))
    recs = (gace_trace_rec * max(n.value, 1))()
    _check(lib().gace_get_trace(ctx, recs, n.value, ctypes.byref(n), ctypes.byref(tpu)))
    dt = np.dtype([("kind", "<u4"), ("index", "<u4"), ("wg", "<u4"), ("xcc", "<u4"), ("t_begin", "<u8"),
                   ("t_ready", "<u8"), ("t_end", "<u8"), ("work", "<u8")])
    arr = np.frombuffer(bytes(recs), dtype=dt, count=n.value).copy()
    return arr, tpu.value


GACE_SERVER_BATCH_COMPLETION = 1


def gace_server_create(device: int = 0, max_inflight: int = 2, max_batch: int = 256,
                       queue_capacity: int = 4096, workspace_bytes: int = 8 << 30, flags: int = 0) -> int:
    cfg = gace_server_cfg()
    cfg.flags = flags
    cfg.max_inflight = max_inflight
    cfg.max_batch = max_batch
    cfg.queue_capacity = queue_capacity
    cfg.workspace_bytes = workspace_bytes
    h = ctypes.c_void_p()
    _check(lib().gace_server_create(device, ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def gace_server_submit(srv: int, req) -> int:
    """Submit one SelRequest / JoinRequest; keeps its ctypes arrays alive on the
    request object until it completes.  Returns the ticket."""
    arr, keep = make_requests([req])
    req._keep = (arr, keep)
    t = ctypes.c_uint64()
    _check(lib().gace_server_submit(srv, arr, ctypes.byref(t)))
    return int(t.value)


def gace_server_wait(srv: int, ticket: int, timeout_ns: int = -1) -> int:
    st = ctypes.c_int32()
    _check(lib().gace_server_wait(srv, ticket, timeout_ns, ctypes.byref(st)))
    return int(st.value)


def gace_server_wait_times(srv: int, ticket: int, timeout_ns: int = -1):
    """(status, submit_ns, done_ns); times are CLOCK_MONOTONIC nanoseconds, the
    clock of time.monotonic_ns()."""
    st = ctypes.c_int32()
    t0 = ctypes.c_uint64()
    t1 = ctypes.c_uint64()
    _check(lib().gace_server_wait_times(srv, ticket, timeout_ns, ctypes.byref(st), ctypes.byref(t0),
                                        ctypes.byref(t1)))
    return int(st.value), int(t0.value), int(t1.value)


def gace_server_submit_raw(srv: int, req_ptr) -> int:
    """Submit a request already marshalled as a gace_request (pointer or
    byref); the caller keeps its arrays alive until it completes."""
    t = ctypes.c_uint64()
    _check(lib().gace_server_submit(srv, req_ptr, ctypes.byref(t)))
    return int(t.value)


def gace_server_stats_get(srv: int) -> dict:
    s = gace_server_stats()
    _check(lib().gace_server_stats_get(srv, ctypes.byref(s)))
    return {n: int(getattr(s, n)) for n, _ in gace_server_stats._fields_}


def gace_server_destroy(srv: int):
    _check(lib().gace_server_destroy(srv))


# ---------------------------------------------------------------- gace_gate.h
def gace_gate_default_cfg() -> gace_gate_cfg:
    c = gace_gate_cfg()
    _check(lib().gace_gate_default_cfg(ctypes.byref(c)))
    return c


def gace_gate_evaluate(cfg: Optional[gace_gate_cfg] = None, ndv=None, sel=None, pcs=None) -> dict:
    """ndv = (ndv_hist, ndv_est); sel = (s_est, count, n); pcs = (c_ab, c_a, c_b, n) or a
    gace_gate_in filled by gace_probe_pcs.  Omitted signals are not evaluated."""
    if cfg is None:
        cfg = gace_gate_default_cfg()
    x = gace_gate_in()
    if ndv is not None:
        x.have |= GATE_DRIFT
        x.ndv_hist, x.ndv_est = float(ndv[0]), float(ndv[1])
    if sel is not None:
        x.have |= GATE_SELERR
        x.s_est, x.count, x.n = float(sel[0]), int(sel[1]), int(sel[2])
    if isinstance(pcs, gace_gate_in):
        x.have |= GATE_PCS
        x.c_ab, x.c_a, x.c_b, x.n_pcs = pcs.c_ab, pcs.c_a, pcs.c_b, pcs.n_pcs
    elif pcs is not None:
        x.have |= GATE_PCS
        x.c_ab, x.c_a, x.c_b, x.n_pcs = (int(v) for v in pcs)
    o = gace_gate_out()
    _check(lib().gace_gate_evaluate(ctypes.byref(cfg), ctypes.byref(x), ctypes.byref(o)))
    return dict(drift=o.drift, sel_err=o.sel_err, pcs=o.pcs, flags=int(o.flags), undefined=int(o.undefined),
                trigger=bool(o.trigger))


def gace_probe_pcs(ctx: int, table: Table, a_terms, b_terms, seed: int = 0, rate: float = 1.0,
                   block_rows: int = 4096, stream=None) -> gace_gate_in:
    """One probe of {A, B, A AND B}; returns the gate inputs (c_ab, c_a, c_b, n_pcs)."""
    keep = _Keep()
    t = _make_table(table, keep)
    p = _make_preds([a_terms, b_terms], [_dtype_code(c) for c in table.cols], keep)
    s = _make_spec(seed, rate, block_rows)
    out = gace_gate_in()
    _check(lib().gace_probe_pcs(ctx, ctypes.byref(t), ctypes.byref(p), ctypes.byref(s), ctypes.byref(out),
                                _stream_handle(stream)))
    return out


def _features(n_rows: float, row_bytes: float, terms: float) -> gace_cost_features:
    f = gace_cost_features()
    f.n_rows, f.row_bytes, f.terms = float(n_rows), float(row_bytes), float(terms)
    return f


def gace_cost_create(prior_ms: float = 0.85, window: int = 4096) -> int:
    h = ctypes.c_void_p()
    _check(lib().gace_cost_create(prior_ms, window, ctypes.byref(h)))
    return h.value


def gace_cost_destroy(m: int):
    _check(lib().gace_cost_destroy(m))


def gace_cost_observe(m: int, n_rows: float, row_bytes: float, terms: float, ms: float):
    f = _features(n_rows, row_bytes, terms)
    _check(lib().gace_cost_observe(m, ctypes.byref(f), ms))


def gace_cost_coef(m: int):
    """-> (coefficients [fixed ms, ms per byte, ms per row-term], observations)"""
    c = (ctypes.c_double * 3)()
    n = ctypes.c_uint32()
    _check(lib().gace_cost_coef(m, c, ctypes.byref(n)))
    return [c[0], c[1], c[2]], int(n.value)


def gace_cost_predict(m: int, n_rows: float, row_bytes: float, terms: float) -> float:
    f = _features(n_rows, row_bytes, terms)
    r = ctypes.c_double()
    _check(lib().gace_cost_predict(m, ctypes.byref(f), ctypes.byref(r)))
    return r.value


def gace_cost_features_of(req) -> Tuple[float, float, float]:
    arr, keep = make_requests([req])
    f = gace_cost_features()
    _check(lib().gace_cost_features_of(arr, ctypes.byref(f)))
    return f.n_rows, f.row_bytes, f.terms


def gace_cost_breakeven(device: int, host: int, row_bytes: float, terms: float) -> float:
    r = ctypes.c_double()
    _check(lib().gace_cost_breakeven(device, host, row_bytes, terms, ctypes.byref(r)))
    return r.value


def gace_cache_create(capacity: int = 1 << 16) -> int:
    h = ctypes.c_void_p()
    _check(lib().gace_cache_create(capacity, ctypes.byref(h)))
    return h.value


def gace_cache_destroy(c: int):
    _check(lib().gace_cache_destroy(c))


def _sel_args(table: Table, preds, seed, rate, block_rows, keep):
    t = _make_table(table, keep)
    p = _make_preds(preds, [_dtype_code(c) for c in table.cols], keep)
    return t, p, _make_spec(seed, rate, block_rows)


def gace_cache_lookup(c: int, table: Table, preds, seed: int = 0, rate: float = 1.0, block_rows: int = 4096):
    """-> (counts, hit mask, n_hit, sampled_rows, kept_blocks); counts of misses are 0."""
    keep = _Keep()
    t, p, s = _sel_args(table, preds, seed, rate, block_rows, keep)
    n = max(len(preds), 1)
    counts = np.zeros(n, dtype=np.uint64)
    hit = np.zeros(n, dtype=np.uint8)
    info = gace_probe_info()
    nh = ctypes.c_uint32()
    _check(lib().gace_cache_lookup(c, ctypes.byref(t), ctypes.byref(p), ctypes.byref(s),
                                   counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                   hit.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(info),
                                   ctypes.byref(nh)))
    k = len(preds)
    return counts[:k], hit[:k].astype(bool), int(nh.value), int(info.sampled_rows), int(info.kept_blocks)


def gace_cache_insert(c: int, table: Table, preds, counts, sampled_rows: int, kept_blocks: int, seed: int = 0,
                      rate: float = 1.0, block_rows: int = 4096):
    keep = _Keep()
    t, p, s = _sel_args(table, preds, seed, rate, block_rows, keep)
    cs = np.zeros(max(len(preds), 1), dtype=np.uint64)
    cs[:len(preds)] = np.asarray(counts, dtype=np.uint64)
    info = gace_probe_info()
    info.sampled_rows, info.kept_blocks = sampled_rows, kept_blocks
    _check(lib().gace_cache_insert(c, ctypes.byref(t), ctypes.byref(p), ctypes.byref(s),
                                   cs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), ctypes.byref(info)))


def gace_cache_invalidate(c: int, table_id: int):
    _check(lib().gace_cache_invalidate(c, table_id))


def gace_cache_stats_get(c: int) -> dict:
    st = gace_cache_stats()
    _check(lib().gace_cache_stats_get(c, ctypes.byref(st)))
    return {n: int(getattr(st, n)) for n, _ in gace_cache_stats._fields_}


def gace_probe_selectivity_cached(ctx: int, c: int, table: Table, preds, seed: int = 0, rate: float = 1.0,
                                  block_rows: int = 4096, stream=None):
    """-> (counts, sampled_rows, kept_blocks, n_hit)"""
    keep = _Keep()
    t, p, s = _sel_args(table, preds, seed, rate, block_rows, keep)
    counts = np.zeros(max(len(preds), 1), dtype=np.uint64)
    info = gace_probe_info()
    nh = ctypes.c_uint32()
    _check(lib().gace_probe_selectivity_cached(ctx, c, ctypes.byref(t), ctypes.byref(p), ctypes.byref(s),
                                               counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                               ctypes.byref(info), ctypes.byref(nh), _stream_handle(stream)))
    return counts[:len(preds)], int(info.sampled_rows), int(info.kept_blocks), int(nh.value)


def gace_join_freq_cached(ctx: int, c: int, R: Keys, S: Keys, stream=None):
    """-> (result dict, hit)"""
    r, s = _make_keys(R), _make_keys(S)
    out = gace_join_result()
    hit = ctypes.c_uint32()
    _check(lib().gace_join_freq_cached(ctx, c, ctypes.byref(r), ctypes.byref(s), ctypes.byref(out),
                                       ctypes.byref(hit), _stream_handle(stream)))
    return _join_dict(out), bool(hit.value)


# ---------------------------------------------------------------- gace_host.h
_NP_DTYPE = {np.dtype(np.int32): I32, np.dtype(np.int64): I64, np.dtype(np.float32): F32}


def gace_probe_selectivity_host(ctx: int, cols, table_id: int, preds, seed: int = 0, rate: float = 1.0,
                                block_rows: int = 4096, key_only: bool = True, chunk_rows: int = 0,
                                gather_threads: int = 0, stream=None):
    """Probe a table held in host memory (cols: C-contiguous numpy arrays of
    equal length).  -> (counts, sampled_rows, kept_blocks, transfer stats dict)"""
    keep = _Keep()
    arr = keep.add((gace_column * max(len(cols), 1))())
    dts = []
    for i, c in enumerate(cols):
        if not c.flags["C_CONTIGUOUS"] or c.dtype not in _NP_DTYPE:
            raise TypeError("host columns must be C-contiguous int32, int64 or float32 arrays")
        arr[i].data = c.ctypes.data
        arr[i].dtype = _NP_DTYPE[c.dtype]
        dts.append(_NP_DTYPE[c.dtype])
    t = gace_table()
    t.n_rows = int(cols[0].shape[0]) if cols else 0
    t.cols = ctypes.cast(arr, ctypes.POINTER(gace_column))
    t.n_cols = len(cols)
    t.table_id = table_id
    p = _make_preds(preds, dts, keep)
    s = _make_spec(seed, rate, block_rows)
    o = gace_host_opts()
    o.key_only, o.chunk_rows, o.gather_threads = (1 if key_only else 0), chunk_rows, gather_threads
    counts = np.zeros(max(len(preds), 1), dtype=np.uint64)
    info = gace_probe_info()
    st = gace_transfer_stats()
    _check(lib().gace_probe_selectivity_host(ctx, ctypes.byref(t), ctypes.byref(p), ctypes.byref(s), ctypes.byref(o),
                                             counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                             ctypes.byref(info), ctypes.byref(st), _stream_handle(stream)))
    stats = {n: getattr(st, n) for n, _ in gace_transfer_stats._fields_ if n != "reserved"}
    return counts[:len(preds)], int(info.sampled_rows), int(info.kept_blocks), stats


# ---------------------------------------------------------------- gace_est.h
def gace_estimate_selectivity(count: int, sampled_rows: int, kept_blocks: int, n_rows: int, rate: float = 1.0,
                              block_rows: int = 4096, seed: int = 0) -> dict:
    info = gace_probe_info()
    info.sampled_rows, info.kept_blocks = sampled_rows, kept_blocks
    sp = _make_spec(seed, rate, block_rows)
    e = gace_sel_estimate()
    _check(lib().gace_estimate_selectivity(count, ctypes.byref(info), n_rows, ctypes.byref(sp), ctypes.byref(e)))
    return {n: getattr(e, n) for n, _ in gace_sel_estimate._fields_}


def gace_estimate_join(res: dict, n_rows_R: int, rate_R: float, n_rows_S: int, rate_S: float,
                       block_rows_R: int = 4096, block_rows_S: int = 4096) -> dict:
    r = gace_join_result()
    for n in JOIN_FIELDS:
        setattr(r, n, int(res[n]))
    sr, ss = _make_spec(0, rate_R, block_rows_R), _make_spec(0, rate_S, block_rows_S)
    e = gace_join_estimate()
    _check(lib().gace_estimate_join(ctypes.byref(r), n_rows_R, ctypes.byref(sr), n_rows_S, ctypes.byref(ss),
                                    ctypes.byref(e)))
    return {n: getattr(e, n) for n, _ in gace_join_estimate._fields_}


# ---------------------------------------------------------------- gace_zone.h
ZONE_ROWS = 4096


def gace_zonemap_build(ctx: int, table: Table, stream=None) -> int:
    keep = _Keep()
    t = _make_table(table, keep)
    h = ctypes.c_void_p()
    _check(lib().gace_zonemap_build(ctx, ctypes.byref(t), ctypes.byref(h), _stream_handle(stream)))
    return h.value


def gace_zonemap_destroy(zm: int):
    _check(lib().gace_zonemap_destroy(zm))


def gace_zonemap_info(zm: int) -> int:
    n = ctypes.c_uint64()
    _check(lib().gace_zonemap_info(zm, ctypes.byref(n)))
    return int(n.value)


def gace_zonemap_read(zm: int, col: int, dtype) -> Tuple[np.ndarray, np.ndarray]:
    """-> (per-zone minima, maxima) of column col, as numpy arrays of dtype."""
    n = gace_zonemap_info(zm)
    lo = np.zeros(max(n, 1), dtype=dtype)
    hi = np.zeros(max(n, 1), dtype=dtype)
    _check(lib().gace_zonemap_read(zm, col, lo.ctypes.data, hi.ctypes.data))
    return lo[:n], hi[:n]


def gace_zonemap_attach(ctx: int, zm: int):
    _check(lib().gace_zonemap_attach(ctx, zm))


def gace_zonemap_detach(ctx: int, zm: int):
    _check(lib().gace_zonemap_detach(ctx, zm))


def gace_server_attach_zonemap(srv: int, zm: int):
    _check(lib().gace_server_attach_zonemap(srv, zm))


def gace_probe_selectivity_zm(ctx: int, table: Table, zm: int, preds, seed: int = 0, rate: float = 1.0,
                              block_rows: int = 4096, stream=None):
    """-> (counts, sampled_rows, kept_blocks, zones_skipped)"""
    keep = _Keep()
    t, p, s = _sel_args(table, preds, seed, rate, block_rows, keep)
    counts = np.zeros(max(len(preds), 1), dtype=np.uint64)
    info = gace_probe_info()
    sk = ctypes.c_uint64()
    _check(lib().gace_probe_selectivity_zm(ctx, ctypes.byref(t), zm, ctypes.byref(p), ctypes.byref(s),
                                           counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                           ctypes.byref(info), ctypes.byref(sk), _stream_handle(stream)))
    return counts[:len(preds)], int(info.sampled_rows), int(info.kept_blocks), int(sk.value)
