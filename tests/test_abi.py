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


def test_view_struct_layouts_match_the_c_compiler(tmp_path):
    # offsets and sizes of the view structs as gcc lays out include/snnc.h,
    # against the binding's ctypes declarations
    views = {"snnc_conn_view": snnc.ConnView, "snnc_p2p_view": snnc.P2PView, "snnc_coll_view": snnc.CollView,
             "snnc_stats_t": snnc.Stats, "snnc_conn_spec": snnc.ConnSpec, "snnc_syn_spec": snnc.SynSpec}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{os.path.join(ROOT, "include", "snnc.h")}"',
             "int main(void) {"]
    for cname, cls in views.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-std=c11", "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in views.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_views_reject_null_arguments_without_a_device():
    L = snnc.lib()
    assert L.snnc_get_connections(None, None) == -1
    assert L.snnc_get_p2p_send(None, None) == -1
    assert L.snnc_get_collective(None, 0, None) == -1
    assert L.snnc_copy_to_host(None, 10, None, 0) == -1
    assert L.snnc_get_image_map(None, 0, 0, None, None, None, None) == -1
