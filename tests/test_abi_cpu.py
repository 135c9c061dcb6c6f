"""The C-ABI library loads and exports every function include/*.h declares;
the ctypes layouts match the header; host-side request validation (no GPU).
"""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import paper_2512_19750_amd as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(g.LIB_PATH):
        from paper_2512_19750_amd import build
        build.build()
    return g.lib()


def _declared_functions():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:gace_status|const char\*)\s+(gace_\w+)\s*\(", src, flags=re.M)))


def test_every_declared_function_is_exported(L):
    names = _declared_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(g.ABI_FUNCTIONS)


def test_struct_layouts():
    assert ctypes.sizeof(g.gace_term) == 80
    assert ctypes.sizeof(g.gace_column) == 16
    assert ctypes.sizeof(g.gace_table) == 24
    assert ctypes.sizeof(g.gace_sample_spec) == 24
    assert ctypes.sizeof(g.gace_keys) == 48
    assert ctypes.sizeof(g.gace_join_result) == 72
    assert ctypes.sizeof(g.gace_schedule) == 32
    assert [f for f, _ in g.gace_schedule._fields_][-2] == "agg_wgs_per_cu"
    assert ctypes.sizeof(g.gace_kernel_stats) == 48


def test_version(L):
    assert "gfx950" in g.gace_version()


class _FakeCol:
    """Stands in for a device tensor: validation reads only pointers and dtypes."""
    def __init__(self, ptr, dtype, n):
        import torch
        self._ptr, self.dtype, self.shape = ptr, dtype, (n,)

    def data_ptr(self):
        return self._ptr


def _sel(preds, dtypes=None, n=1000, rate=1.0, block_rows=4096, ptr=0x10000):
    import torch
    td = {1: torch.int32, 2: torch.int64, 3: torch.float32}
    dtypes = dtypes or [1, 1, 2, 3]
    cols = [_FakeCol(ptr + 0x1000 * i, td[d], n) for i, d in enumerate(dtypes)]
    return g.SelRequest(g.Table(cols, 1), preds, seed=1, rate=rate, block_rows=block_rows)


def test_check_request_accepts_valid(L):
    r = _sel([[(0, g.RANGE, (1, 5)), (3, g.RANGE, (0.0, 1.0))], [(2, g.IN, (1, 2, 3))]])
    assert g.gace_check_request(r) == g.GACE_OK


@pytest.mark.parametrize("bad", [
    [[]],                                                         # predicate with no terms
    [[(0, g.RANGE, (1, 5))] * 17],                                # > 16 terms
    [[(9, g.EQ, (1,))]],                                          # column out of range
    [[(0, g.RANGE, (1,))]],                                       # RANGE with one value
    [[(0, g.EQ, (1, 2))]],                                        # EQ with two values
    [[(0, g.IN, tuple(range(9)))]],                               # IN with 9 values
    [[(3, g.RANGE, (float("nan"), 1.0))]],                        # NaN float bound
    [[(0, 7, (1,))]],                                             # unknown op
])
def test_check_request_rejects(L, bad):
    assert g.gace_check_request(_sel(bad)) == g.GACE_EINVAL
    assert g.last_error()


@pytest.mark.parametrize("rate,block_rows", [(-0.1, 4096), (1.5, 4096), (float("nan"), 4096), (0.5, 3000),
                                             (0.5, 0), (0.5, 1 << 21)])
def test_check_request_rejects_specs(L, rate, block_rows):
    r = _sel([[(0, g.EQ, (1,))]], rate=rate, block_rows=block_rows)
    assert g.gace_check_request(r) == g.GACE_EINVAL


def test_check_request_rejects_misaligned_column(L):
    assert g.gace_check_request(_sel([[(0, g.EQ, (1,))]], ptr=0x10004)) == g.GACE_EINVAL


def test_check_join(L):
    class K:
        def __init__(self, ptr, n):
            self._p, self.shape = ptr, (n,)

        def data_ptr(self):
            return self._p
    ok = g.JoinRequest(g.Keys(K(0x1000, 100), 1), g.Keys(K(0x2000, 100), 2))
    assert g.gace_check_request(ok) == g.GACE_OK
    big = g.JoinRequest(g.Keys(K(0x1000, 2**32 - 1), 1), g.Keys(K(0x2000, 2**32 - 1), 2, rate=0.5))
    assert g.gace_check_request(big) == g.GACE_OK
    huge = g.JoinRequest(g.Keys(K(0x1000, 2**32), 1), g.Keys(K(0x2000, 10), 2))
    assert g.gace_check_request(huge) == g.GACE_EINVAL
    mis = g.JoinRequest(g.Keys(K(0x1004, 10), 1), g.Keys(K(0x2000, 10), 2))
    assert g.gace_check_request(mis) == g.GACE_EINVAL
    null = g.JoinRequest(g.Keys(K(0, 10), 1), g.Keys(K(0x2000, 10), 2))
    assert g.gace_check_request(null) == g.GACE_EINVAL


def test_struct_sizes_match_the_c_headers(tmp_path):
    """Every ctypes mirror has the size the C compiler gives the header's struct."""
    import subprocess
    names = ["gace_term", "gace_column", "gace_table", "gace_sample_spec", "gace_keys", "gace_join_result",
             "gace_request", "gace_probe_info", "gace_schedule", "gace_kernel_stats", "gace_server_cfg",
             "gace_server_stats"]
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include "gace.h"\n#include "gace_zone.h"\nint main(void) {\n' +
                   "".join('    printf("%%s %%zu\\n", "%s", sizeof(%s));\n' % (n, n) for n in names) +
                   "    return 0;\n}\n")
    exe = tmp_path / "sizes"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    c_sizes = dict(zip(out[::2], (int(x) for x in out[1::2])))
    for n in names:
        assert ctypes.sizeof(getattr(g, n)) == c_sizes[n], n
