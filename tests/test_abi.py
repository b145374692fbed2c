"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the header declares, rejects bad arguments before touching a
device, and builds the same delay tables as the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2512_09502_amd as snnc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "snnc.h")).read()
    return sorted(set(re.findall(r"^(?:snnc_status|const char\*)\s+(snnc_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    L = snnc.lib()
    declared = _declared()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(L, name), f"{name} declared in snnc.h but not exported"
    assert sorted(snnc.EXPORTS) == declared


def test_init_rejects_bad_arguments_without_a_device():
    L = snnc.lib()
    h = ctypes.c_void_p()
    assert L.snnc_init(ctypes.byref(h), 0, 0, 1, 0.1, None, None, 0) == -1      # P = 0
    assert L.snnc_init(ctypes.byref(h), 2, 2, 1, 0.1, None, None, 0) == -1      # P_local >= P
    assert L.snnc_init(ctypes.byref(h), 2, 0, 1, 0.0, None, None, 0) == -1      # dt <= 0
    assert L.snnc_init(None, 2, 0, 1, 0.1, None, None, 0) == -1


@pytest.mark.parametrize("mean,sd,lo,dt", [(1.5, 0.75, 0.1, 0.1), (3.0, 1.5, 0.1, 0.1), (0.5, 2.0, 0.3, 0.1),
                                           (10.0, 0.05, 0.1, 0.1), (2.0, 1.0, 0.25, 0.05), (50.0, 20.0, 1.0, 0.1)])
def test_delay_tables_identical_to_oracle(mean, sd, lo, dt):
    a = snnc.delay_table(mean, sd, lo, dt)
    b = oracle.delay_table(mean, sd, lo, dt)
    assert a is not None and b is not None
    assert a[0] == b[0]
    np.testing.assert_array_equal(a[1], b[1])


def test_delay_table_rejections_match_oracle():
    for args in [(7000.0, 1.0, 0.1, 0.1), (1.0, 1.0, 0.04, 0.1)]:
        assert snnc.delay_table(*args) is None
        assert oracle.delay_table(*args) is None


def test_struct_layouts_match_header():
    # sizes of the ABI structs as laid out by the C compiler on this platform
    assert ctypes.sizeof(snnc.Segment) == 12
    assert ctypes.sizeof(snnc.ConnSpec) == 32
    assert ctypes.sizeof(snnc.Dist) == 32
    assert ctypes.sizeof(snnc.SynSpec) == 72
    assert ctypes.sizeof(snnc.Stats) == 64
