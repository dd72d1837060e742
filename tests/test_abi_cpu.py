"""CPU-side checks of the C ABI: the library loads and exports what the header declares."""
import ctypes
import os
import subprocess

import pytest

from conftest import ROOT, header_functions
from paper_2208_04514_amd import dawn as D


def test_library_exports_every_header_function(dawn_lib):
    declared = header_functions()
    assert len(declared) >= 16
    for name in declared:
        assert hasattr(dawn_lib, name), f"{name} declared in dawn.h but not exported"
    assert set(declared) == set(D.EXPORTED)


def test_binding_names_match_header():
    for name in header_functions():
        assert callable(getattr(D, name)), f"binding lacks {name}"


def test_null_context_rejected(dawn_lib):
    st = dawn_lib.dawn_sssp(None, 0, 0, None, 0, None)
    assert st == D.DAWN_E_INVALID_ARG
    assert dawn_lib.dawn_destroy(None) == D.DAWN_E_INVALID_ARG
    assert "null" in D.dawn_last_error()


def test_struct_layouts_match_header():
    # offsets the C compiler gives the public structs must match the ctypes mirrors
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "dawn.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(dawn_run_stats), offsetof(dawn_run_stats, frontier_cap),
         offsetof(dawn_run_stats, kernel_clock_ms));
  printf("%zu %zu %zu %zu\n",
         sizeof(dawn_params), offsetof(dawn_params, timing),
         offsetof(dawn_params, small_frontier_edges), offsetof(dawn_params, medium_groups));
  printf("%zu %zu %zu %zu\n", sizeof(dawn_graph_info), offsetof(dawn_graph_info, device_bytes),
         sizeof(dawn_query_stats), offsetof(dawn_query_stats, batch_peak));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    got = list(map(int, out))
    want = [ctypes.sizeof(D.RunStats), D.RunStats.frontier_cap.offset,
            D.RunStats.kernel_clock_ms.offset, ctypes.sizeof(D.Params), D.Params.timing.offset,
            D.Params.small_frontier_edges.offset, D.Params.medium_groups.offset,
            ctypes.sizeof(D.GraphInfo), D.GraphInfo.device_bytes.offset,
            ctypes.sizeof(D.QueryStats), D.QueryStats.batch_peak.offset]
    assert got == want


def test_output_buffers_checked_before_any_call():
    """A buffer that does not hold exactly what the call writes is refused by
    the binding (the C ABI has no length argument to catch it)."""
    import numpy as np
    ptr, flags, _ = D.check_out(np.empty((3, 5), np.int32), (3, 5))
    assert flags == 0 and ptr
    D.check_out(np.empty(15, np.int32), (3, 5))           # flat of the same size
    bad = [np.empty((2, 5), np.int32),                    # too short
           np.empty((3, 6), np.int32),                    # too long
           np.empty((5, 3), np.int32),                    # same size, other shape
           np.empty((3, 5), np.int64),                    # wrong dtype
           np.empty((5, 3), np.int32).T,                  # not C-contiguous
           [0] * 15]
    for b in bad:
        with pytest.raises(ValueError):
            D.check_out(b, (3, 5))
    ro = np.empty((3, 5), np.int32)
    ro.flags.writeable = False
    with pytest.raises(ValueError):
        D.check_out(ro, (3, 5))
