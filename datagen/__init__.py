"""Seeded synthetic inputs for the probe workloads.

This package is the only code that both the oracle side and the device side
use.  It contains the counter-based column generator (gen_core.h, with a host
fill in C and a device fill in HIP) and the workload recipes: table shapes,
column laws, predicate sets and sampling specs.  It holds none of the probe
method's arithmetic: no sampler, no predicate evaluation, no counting and no
key aggregation.

Predicates are plain Python data: a predicate is a list of terms
``(col, op, values)`` with ``op`` one of RANGE / EQ / IN.  A RANGE term is
``values = (lo, hi)`` meaning ``lo <= x < hi``; for float columns the values
are Python floats.  The oracle and the device binding each marshal this into
their own C structures.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
HOST_LIB = os.path.join(HERE, "libgacegen_host.so")
DEV_LIB = os.path.join(HERE, "libgacegen_dev.so")

# seeds: workload k uses S0+k for data, S0+16+k for predicates, S0+32+k for sampling
S0 = 0x2512197500

UNIFORM, ZIPF, F32UNIT = 1, 2, 3
I32, I64, F32 = 1, 2, 3
RANGE, EQ, IN = 1, 2, 3

DTYPE_NP = {I32: np.int32, I64: np.int64, F32: np.float32}
DTYPE_BYTES = {I32: 4, I64: 8, F32: 4}


# ----------------------------------------------------------------------------
# build + load
# ----------------------------------------------------------------------------
HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build_host() -> str:
    cmd = ["gcc", "-O2", "-Wall", "-fPIC", "-shared", "-o", HOST_LIB,
           os.path.join(HERE, "gen_host.c"), "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    return HOST_LIB


def build_device() -> str:
    cmd = ["/opt/rocm/bin/hipcc", *HIP_FLAGS, "-o", DEV_LIB, os.path.join(HERE, "gen_dev.hip")]
    subprocess.run(cmd, check=True)
    return DEV_LIB


class GgCol(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("dtype", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("lo", ctypes.c_int64), ("span", ctypes.c_uint64),
                ("cdf", ctypes.c_void_p), ("ncdf", ctypes.c_uint64),
                ("noise_seed", ctypes.c_uint64), ("noise_lo", ctypes.c_int64),
                ("noise_span", ctypes.c_uint64)]


_host = None
_dev = None


def host_lib():
    global _host
    if _host is None:
        if not os.path.exists(HOST_LIB):
            build_host()
        lib = ctypes.CDLL(HOST_LIB)
        lib.gg_zipf_cdf.argtypes = [ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p]
        lib.gg_zipf_cdf.restype = ctypes.c_int
        lib.gg_stream_seed_host.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        lib.gg_stream_seed_host.restype = ctypes.c_uint64
        lib.gg_fill_host.argtypes = [ctypes.POINTER(GgCol), ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_void_p, ctypes.c_int]
        lib.gg_fill_host.restype = ctypes.c_int
        lib.gg_values_at.argtypes = [ctypes.POINTER(GgCol), ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        lib.gg_values_at.restype = ctypes.c_int
        _host = lib
    return _host


def dev_lib():
    global _dev
    if _dev is None:
        import torch  # noqa: F401  (the HIP runtime torch loaded is the one this library binds to)
        if not os.path.exists(DEV_LIB):
            build_device()
        lib = ctypes.CDLL(DEV_LIB)
        lib.gg_fill_device.argtypes = [ctypes.POINTER(GgCol), ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_fill_device.restype = ctypes.c_int
        _dev = lib
    return _dev


def stream_seed(seed: int, table: int, col: int, draw: int = 0) -> int:
    return int(host_lib().gg_stream_seed_host(seed & (2**64 - 1), table, col, draw))


_CDF_CACHE = {}


def zipf_cdf(s: float, n: int) -> np.ndarray:
    key = (float(s), int(n))
    if key not in _CDF_CACHE:
        out = np.empty(int(n), dtype=np.uint64)
        if host_lib().gg_zipf_cdf(float(s), int(n), out.ctypes.data) != 0:
            raise ValueError("bad zipf parameters")
        _CDF_CACHE[key] = out
    return _CDF_CACHE[key]


# ----------------------------------------------------------------------------
# column + table specs
# ----------------------------------------------------------------------------
@dataclass
class ColSpec:
    dtype: int
    kind: int
    seed: int                    # user seed; stream seed derives from (seed, table, col)
    table: int
    col: int
    lo: int = 0
    span: int = 1
    zipf_s: float = 0.0
    zipf_n: int = 0
    noise_lo: int = 0
    noise_span: int = 0
    base_col: Optional[int] = None   # draw the base law from this column's stream (correlated columns)

    def cstruct(self, cdf_ptr: Optional[int] = None) -> GgCol:
        base = self.col if self.base_col is None else self.base_col
        c = GgCol()
        c.kind = self.kind
        c.dtype = self.dtype
        c.seed = stream_seed(self.seed, self.table, base, 0)
        c.lo = self.lo
        c.span = self.span
        c.cdf = cdf_ptr or 0
        c.ncdf = self.zipf_n if self.kind == ZIPF else 0
        c.noise_seed = stream_seed(self.seed, self.table, self.col, 1) if self.noise_span else 0
        c.noise_lo = self.noise_lo
        c.noise_span = self.noise_span
        return c

    @property
    def nbytes_per_row(self) -> int:
        return DTYPE_BYTES[self.dtype]


@dataclass
class TableSpec:
    n_rows: int
    cols: List[ColSpec]
    table_id: int

    @property
    def row_bytes(self) -> int:
        return sum(c.nbytes_per_row for c in self.cols)


@dataclass
class SampleSpec:
    seed: int
    rate: float
    block_rows: int = 4096


Term = Tuple[int, int, tuple]         # (col, op, values)
Predicate = List[Term]


@dataclass
class SelRequest:
    table: int                         # index into the workload's table list
    preds: List[Predicate]
    spec: SampleSpec


@dataclass
class JoinRequest:
    r: TableSpec                       # one i64 key column each
    s: TableSpec
    spec_r: SampleSpec
    spec_s: SampleSpec


@dataclass
class Workload:
    name: str
    tables: List[TableSpec] = field(default_factory=list)
    sel: List[SelRequest] = field(default_factory=list)
    joins: List[JoinRequest] = field(default_factory=list)
    order: List[Tuple[str, int]] = field(default_factory=list)   # batch order: ("sel", i) / ("join", j)


# ----------------------------------------------------------------------------
# host / device materialisation
# ----------------------------------------------------------------------------
def host_column(c: ColSpec, n: int, row0: int = 0, nthreads: int = 8) -> np.ndarray:
    out = np.empty(int(n), dtype=DTYPE_NP[c.dtype])
    cdf = zipf_cdf(c.zipf_s, c.zipf_n) if c.kind == ZIPF else None
    cs = c.cstruct(cdf.ctypes.data if cdf is not None else None)
    if host_lib().gg_fill_host(ctypes.byref(cs), int(row0), int(n), out.ctypes.data, int(nthreads)) != 0:
        raise ValueError("gg_fill_host failed")
    return out


def host_values_at(c: ColSpec, rows: np.ndarray) -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    out = np.empty(rows.shape[0], dtype=np.int64)
    cdf = zipf_cdf(c.zipf_s, c.zipf_n) if c.kind == ZIPF else None
    cs = c.cstruct(cdf.ctypes.data if cdf is not None else None)
    if host_lib().gg_values_at(ctypes.byref(cs), rows.ctypes.data, rows.shape[0], out.ctypes.data) != 0:
        raise ValueError("gg_values_at failed")
    return out


def host_table(t: TableSpec, row0: int = 0, n: Optional[int] = None, nthreads: int = 8) -> List[np.ndarray]:
    n = t.n_rows - row0 if n is None else n
    return [host_column(c, n, row0, nthreads) for c in t.cols]


def device_column(c: ColSpec, n: int, device="cuda", row0: int = 0):
    """Generate n rows of column c directly into a new device tensor."""
    import torch
    tdt = {I32: torch.int32, I64: torch.int64, F32: torch.float32}[c.dtype]
    out = torch.empty(int(n), dtype=tdt, device=device)
    cdf_dev = None
    if c.kind == ZIPF:
        cdf_dev = torch.from_numpy(zipf_cdf(c.zipf_s, c.zipf_n).view(np.int64)).to(device)
    cs = c.cstruct(cdf_dev.data_ptr() if cdf_dev is not None else None)
    stream = torch.cuda.current_stream(out.device).cuda_stream
    if n and dev_lib().gg_fill_device(ctypes.byref(cs), int(row0), int(n), out.data_ptr(), stream) != 0:
        raise RuntimeError("gg_fill_device failed")
    if cdf_dev is not None:
        torch.cuda.current_stream(out.device).synchronize()
        del cdf_dev
    return out


def device_table(t: TableSpec, device="cuda"):
    return [device_column(c, t.n_rows, device) for c in t.cols]


# ----------------------------------------------------------------------------
# predicate generation (term law shared by the selectivity workloads)
# ----------------------------------------------------------------------------
def f32_bits(x: float) -> int:
    return int(np.array([x], dtype=np.float32).view(np.uint32)[0])


def bits_f32(b: int) -> float:
    return float(np.array([b & 0xFFFFFFFF], dtype=np.uint32).view(np.float32)[0])


def _draw_values(rng: np.random.Generator, c: ColSpec, n_rows: int, k: int):
    rows = rng.integers(0, n_rows, size=k, dtype=np.uint64)
    v = host_values_at(c, rows)
    if c.dtype == F32:
        return [bits_f32(int(x)) for x in v]
    return [int(x) for x in v]


def random_predicates(rng: np.random.Generator, t: TableSpec, n_preds: int,
                      cols: Optional[Sequence[int]] = None, min_terms: int = 2,
                      max_terms: int = 4) -> List[Predicate]:
    """Each predicate: U{min..max} terms on distinct columns.  Float columns get
    RANGE terms; integer columns RANGE (50 %), EQ (25 %) or IN (25 %, list length
    U{2..8}).  Bounds and values are drawn from the column's own generator at
    random rows, so skewed columns get their heavy values."""
    cols = list(range(len(t.cols))) if cols is None else list(cols)
    preds = []
    for _ in range(n_preds):
        k = int(rng.integers(min_terms, max_terms + 1))
        k = min(k, len(cols))
        chosen = rng.choice(np.array(cols), size=k, replace=False)
        terms = []
        for ci in sorted(int(x) for x in chosen):
            c = t.cols[ci]
            if c.dtype == F32:
                a, b = _draw_values(rng, c, t.n_rows, 2)
                terms.append((ci, RANGE, (min(a, b), max(a, b))))
                continue
            u = rng.random()
            if u < 0.5:
                a, b = _draw_values(rng, c, t.n_rows, 2)
                terms.append((ci, RANGE, (min(a, b), max(a, b) + 1)))
            elif u < 0.75:
                terms.append((ci, EQ, tuple(_draw_values(rng, c, t.n_rows, 1))))
            else:
                m = int(rng.integers(2, 9))
                terms.append((ci, IN, tuple(_draw_values(rng, c, t.n_rows, m))))
        preds.append(terms)
    return preds


# ----------------------------------------------------------------------------
# workload recipes
# ----------------------------------------------------------------------------
def uniform_i32_table(n_rows: int, n_cols: int, seed: int, table_id: int, lo=0, hi=1000) -> TableSpec:
    return TableSpec(n_rows, [ColSpec(I32, UNIFORM, seed, table_id, c, lo=lo, span=hi - lo)
                              for c in range(n_cols)], table_id)


def config1(n_rows: int = 1_000_000) -> Workload:
    """One table of n rows x 4 int32 columns U[0,1000); predicate
    c0 in [100,300) AND c1 in [0,500); full scan (rate 1)."""
    t = uniform_i32_table(n_rows, 4, S0 + 1, table_id=1)
    pred = [(0, RANGE, (100, 300)), (1, RANGE, (0, 500))]
    w = Workload("plain single probe: %d rows x 4 i32 U[0,1000), 1 predicate, rate 1" % n_rows, tables=[t])
    w.sel.append(SelRequest(0, [pred], SampleSpec(S0 + 33, 1.0, 4096)))
    w.order = [("sel", 0)]
    return w


def config2_table(n_rows: int = 100_000_000) -> TableSpec:
    seed, tid = S0 + 2, 2
    cols = [
        ColSpec(I32, ZIPF, seed, tid, 0, lo=0, zipf_s=1.1, zipf_n=1_000_000),
        ColSpec(I32, ZIPF, seed, tid, 1, lo=0, zipf_s=1.1, zipf_n=1_000_000,
                noise_lo=-50, noise_span=101, base_col=0),
        ColSpec(I32, ZIPF, seed, tid, 2, lo=0, zipf_s=1.3, zipf_n=10_000),
        ColSpec(I32, UNIFORM, seed, tid, 3, lo=0, span=1_000_000),
        ColSpec(I64, UNIFORM, seed, tid, 4, lo=0, span=1_000_000),
        ColSpec(I64, UNIFORM, seed, tid, 5, lo=-(1 << 40), span=1 << 41),
        ColSpec(F32, F32UNIT, seed, tid, 6),
        ColSpec(F32, F32UNIT, seed, tid, 7),
    ]
    return TableSpec(n_rows, cols, tid)


def config2(n_rows: int = 100_000_000, n_preds: int = 64, rate: float = 0.01) -> Workload:
    """Skewed correlated multi-predicate probe: 8 columns (Zipf 1.1, Zipf 1.1 +
    U{-50..50}, Zipf 1.3, uniform i32, uniform i64, wide uniform i64, two
    uniform f32); 64 predicates of 2-4 terms; block-Bernoulli 1 %, 4096-row
    blocks."""
    t = config2_table(n_rows)
    rng = np.random.default_rng(S0 + 18)
    preds = random_predicates(rng, t, n_preds)
    w = Workload("skewed correlated multi-predicate probe: %d rows x 8 cols, %d predicates, rate %g"
                 % (n_rows, n_preds, rate), tables=[t])
    w.sel.append(SelRequest(0, preds, SampleSpec(S0 + 34, rate, 4096)))
    w.order = [("sel", 0)]
    return w


def join_pair(n_r: int, n_s: int, domain: int, seed: int, tid_r: int, tid_s: int,
              zipf_s: float = 1.0) -> Tuple[TableSpec, TableSpec]:
    r = TableSpec(n_r, [ColSpec(I64, ZIPF, seed, tid_r, 0, lo=0, zipf_s=zipf_s, zipf_n=domain)], tid_r)
    s = TableSpec(n_s, [ColSpec(I64, UNIFORM, seed, tid_s, 0, lo=0, span=domain)], tid_s)
    return r, s


def config3(rate: float = 1.0, n_r: int = 200_000_000, n_s: int = 50_000_000,
            domain: int = 10_000_000) -> Workload:
    """Join-key frequency probe: R Zipf(1.0) over the domain, S uniform over it."""
    r, s = join_pair(n_r, n_s, domain, S0 + 3, 3, 4)
    w = Workload("join-key frequency probe: R %d Zipf(1.0), S %d uniform, domain %d, rate %g"
                 % (n_r, n_s, domain, rate))
    w.joins.append(JoinRequest(r, s, SampleSpec(S0 + 35, rate, 4096), SampleSpec(S0 + 36, rate, 4096)))
    w.order = [("join", 0)]
    return w


def config4(scale: float = 1.0, n_tables: int = 16, n_sel: int = 448, n_join: int = 64,
            min_rows: int = 1_000_000, max_rows: int = 500_000_000, seed_offset: int = 0) -> Workload:
    """Batched uneven probes: tables with log-uniform row counts in
    [min_rows, max_rows] x 4 i32 U[0,1000); n_sel selectivity requests (table
    uniform, 1-32 predicates, rate log-uniform [0.1 %, 100 %], one sampling seed
    per table) and n_join join probes of the join-probe shape scaled by
    log-uniform [0.01, 1] (rate 1 or 0.05).  `scale` shrinks every size for
    tests."""
    rng = np.random.default_rng(S0 + 20 + seed_offset)
    w = Workload("batched uneven probes: %d sel requests over %d tables + %d joins (scale %g)"
                 % (n_sel, n_tables, n_join, scale))
    lo, hi = math.log(min_rows), math.log(max_rows)
    for t in range(n_tables):
        n = max(1, int(round(math.exp(rng.uniform(lo, hi)) * scale)))
        w.tables.append(uniform_i32_table(n, 4, S0 + 4 + seed_offset, table_id=100 + t))
    table_seeds = [S0 + 1000 + 7 * t + seed_offset for t in range(n_tables)]
    for _ in range(n_sel):
        ti = int(rng.integers(0, n_tables))
        p = int(rng.integers(1, 33))
        preds = random_predicates(rng, w.tables[ti], p)
        rate = float(math.exp(rng.uniform(math.log(0.001), 0.0)))
        w.sel.append(SelRequest(ti, preds, SampleSpec(table_seeds[ti], rate, 4096)))
    for j in range(n_join):
        s = float(math.exp(rng.uniform(math.log(0.01), 0.0)))
        n_r = max(1, int(round(200_000_000 * s * scale)))
        n_s = max(1, int(round(50_000_000 * s * scale)))
        dom = max(1, int(round(10_000_000 * s * scale)))
        r, sd = join_pair(n_r, n_s, dom, S0 + 5000 + 13 * j + seed_offset, 1000 + 2 * j, 1001 + 2 * j)
        rate = 1.0 if rng.random() < 0.5 else 0.05
        w.joins.append(JoinRequest(r, sd, SampleSpec(S0 + 9000 + 2 * j, rate, 4096),
                                   SampleSpec(S0 + 9001 + 2 * j, rate, 4096)))
    order = [("sel", i) for i in range(n_sel)] + [("join", j) for j in range(n_join)]
    perm = rng.permutation(len(order))
    w.order = [order[i] for i in perm]
    return w


def config5(scale: float = 1.0, target_bytes: float = 170e9, n_pool: int = 2048,
            seed_offset: int = 0) -> Workload:
    """Served probe stream: tables drawn from config 4's size law (log-uniform
    1e6..5e8 rows x 4 i32 U[0,1000)) until they hold target_bytes (x scale),
    config 4's 64 join-key pairs, and a pool of n_pool requests drawn from
    config 4's mix (448 selectivity : 64 join) over them.  `order` is the pool;
    a join pair may appear in it several times."""
    rng = np.random.default_rng(S0 + 25 + seed_offset)
    w4 = config4(scale=scale, seed_offset=seed_offset)
    w = Workload("served probe stream: tables of config 4's size law up to %.3g bytes + 64 join pairs, "
                 "pool of %d requests (scale %g)" % (target_bytes * scale, n_pool, scale))
    lo, hi = math.log(1_000_000), math.log(500_000_000)
    total = 0
    while total < target_bytes * scale:
        n = max(1, int(round(math.exp(rng.uniform(lo, hi)) * scale)))
        w.tables.append(uniform_i32_table(n, 4, S0 + 5 + seed_offset, table_id=2000 + len(w.tables)))
        total += n * 16
    w.joins = w4.joins
    table_seeds = [S0 + 3000 + 7 * t + seed_offset for t in range(len(w.tables))]
    for _ in range(n_pool):
        if rng.random() < 64.0 / 512.0:
            w.order.append(("join", int(rng.integers(0, len(w.joins)))))
            continue
        ti = int(rng.integers(0, len(w.tables)))
        p = int(rng.integers(1, 33))
        preds = random_predicates(rng, w.tables[ti], p)
        rate = float(math.exp(rng.uniform(math.log(0.001), 0.0)))
        w.sel.append(SelRequest(ti, preds, SampleSpec(table_seeds[ti], rate, 4096)))
        w.order.append(("sel", len(w.sel) - 1))
    return w


def workload_bytes(w: Workload) -> int:
    tb = sum(t.n_rows * t.row_bytes for t in w.tables)
    jb = sum((j.r.n_rows + j.s.n_rows) * 8 for j in w.joins)
    return tb + jb


def materialise(w: Workload, device="cuda"):
    """Generate every table and join key array of a workload in device memory."""
    tabs = [device_table(t, device) for t in w.tables]
    keys = [(device_column(j.r.cols[0], j.r.n_rows, device), device_column(j.s.cols[0], j.s.n_rows, device))
            for j in w.joins]
    return tabs, keys
