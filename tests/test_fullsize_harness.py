"""CPU checks of the full-size parity harness (tests/fullsize_oracle.py)
against the plain oracle's whole run: on small networks, the harness's
chunked, multi-process reassembly -- sorted connections per source' range,
row counts, image map, point-to-point send lists and collective arrays --
equals the oracle's own arrays exactly, and a planted difference in the
compared arrays is reported."""
import os

import numpy as np
import pytest

import oracle
from fullsize_oracle import FullSizeOracle
from paper_2512_09502_amd import workloads as W

ARRAYS = ("src", "tgt", "delay", "weight", "row_ptr")


def _dump(ref, d):
    os.makedirs(d, exist_ok=True)
    for name in ARRAYS:
        np.save(os.path.join(d, f"{name}.npy"), ref.array(name))


def _harness(script, P_local, tmp_path, **kw):
    ref = oracle.run_script(script, P_local, skip_invalid=True)
    drop = {k for k, _ in ref.rejected}
    calls = [op for k, op in enumerate(script["ops"]) if op[0] == "connect" and k not in drop]
    h = FullSizeOracle(script, P_local, calls, str(tmp_path / "work"), workers=2, log=lambda *_: None,
                       item_records=kw.pop("item_records", 700), task_records=kw.pop("task_records", 900), **kw)
    return ref, h


SCRIPTS = [
    ("balanced", lambda: W.balanced_small(), 0),
    ("column", lambda: W.column8(scale=0.01), 0),
    ("multiarea", lambda: W.multiarea_p2p(P=4, n_e=120, n_i=30, k_e=12, k_i=4, k_remote_max=6, seed=5), 0),
    ("multiarea_h2", lambda: W.multiarea_p2p(P=4, n_e=120, n_i=30, k_e=12, k_i=4, k_remote_max=6, seed=5), 2),
    ("collective", lambda: W.balanced_collective(P=6, n_e=80, n_i=20, k_e=9, k_i=3), 0),
    ("collective_h3", lambda: W.balanced_collective(P=6, n_e=80, n_i=20, k_e=9, k_i=3), 3),
    ("tiny7", lambda: W.random_tiny(7, P=3), 1),
    ("tiny12", lambda: W.random_tiny(12, P=2), 0),
]


@pytest.mark.parametrize("name,make,P_local", SCRIPTS, ids=[s[0] for s in SCRIPTS])
def test_harness_equals_whole_oracle_run(name, make, P_local, tmp_path):
    script = make()
    ref, h = _harness(script, P_local, tmp_path)
    try:
        h.generate()
        assert h.n_generated == ref.array("src").size
        gpu = tmp_path / "gpu"
        _dump(ref, gpu)
        n, errors = h.compare(str(gpu))
        assert errors == [] and n == ref.array("src").size
        m = h.image_map()
        for k in ("r_off", "r_val", "l_val", "img_base"):
            np.testing.assert_array_equal(m[k], ref.array(k), err_msg=k)
        if name.startswith("multiarea"):
            sl = h.send_lists()
            for k in ("s_off", "s_val", "tp_ptr", "t_val", "p_val"):
                np.testing.assert_array_equal(sl[k], ref.array(k), err_msg=k)
        if name.startswith("collective") or name.startswith("tiny"):
            co = h.collective()
            for k in ("groups", "h_off", "h_val", "i_val", "gq_ptr", "g_val", "q_val"):
                np.testing.assert_array_equal(co[k], ref.array(k), err_msg=k)
    finally:
        h.close()


def test_harness_reports_a_planted_difference(tmp_path):
    script = W.multiarea_p2p(P=3, n_e=100, n_i=20, k_e=10, k_i=3, k_remote_max=5, seed=2)
    ref, h = _harness(script, 0, tmp_path)
    try:
        h.generate()
        gpu = tmp_path / "gpu"
        _dump(ref, gpu)
        for name, edit in (("tgt", lambda a: a.__setitem__(777, a[777] + 1)),
                           ("weight", lambda a: a.__setitem__(5, np.nextafter(np.nextafter(np.nextafter(
                               a[5], np.float32(9)), np.float32(9)), np.float32(9)))),
                           ("row_ptr", lambda a: a.__setitem__(40, a[40] + 1))):
            a = ref.array(name)
            edit(a)
            np.save(os.path.join(gpu, f"{name}.npy"), a)
            _, errors = h.compare(str(gpu))
            assert errors, f"a changed {name} went unnoticed"
            np.save(os.path.join(gpu, f"{name}.npy"), ref.array(name))
        assert h.compare(str(gpu))[1] == []
    finally:
        h.close()


def test_harness_rows_and_counts_one_host(tmp_path):
    script = W.served_requests(n_requests=40, n_pops=6, pop_min=50, pop_max=400, size_min=10, size_max=3000, seed=4)
    ref = oracle.run_script(script, 0, skip_invalid=True)
    drop = {k for k, _ in ref.rejected}
    calls = [op for k, op in enumerate(script["ops"]) if op[0] == "connect" and k not in drop]
    M = ref.array("row_ptr").size - 1
    rng = np.random.default_rng(1)
    select = np.zeros(M, bool)
    select[rng.choice(M, size=M // 5, replace=False)] = True
    h = FullSizeOracle(script, 0, calls, str(tmp_path / "work"), workers=2, select=select, row_counts=True,
                       log=lambda *_: None, item_records=500, task_records=300)
    try:
        h.generate()
        rp = ref.array("row_ptr").astype(np.int64)
        np.testing.assert_array_equal(h.rows, np.diff(rp))
        gpu = tmp_path / "gpu"
        _dump(ref, gpu)
        n, errors = h.compare(str(gpu))
        assert errors == [] and n == int(np.diff(rp)[select].sum())
    finally:
        h.close()


def test_served_admission_equals_sequential_definition():
    # the parallel, id-predicting admission equals request-by-request admission
    # (count under the next call id, admit if it fits the budget)
    from fullsize_oracle import connect_ops, meta_bytes, served_admission, validate_requests
    script = W.served_requests(n_requests=70, n_pops=8, pop_min=60, pop_max=500, size_min=10, size_max=4e4, seed=6)
    budget = 14 * 150_000 + 20_000
    status, admitted, counts = served_admission(script, budget, workers=2, pairs_per_job=5000)
    ops = connect_ops(script)
    valid = validate_requests(script)
    net = oracle.OracleNet(1, 0, script["seed"], script["dt"])
    for op in script["ops"]:
        if op[0] == "create":
            net.create(op[1], op[2])
    want_status, want_adm, want_counts, resident = [], [], [], 0
    for k, op in enumerate(ops):
        if valid[k] != 0:
            want_status.append(valid[k])
            continue
        _, src, tgt, conn, syn, alpha = op
        probe = oracle.OracleNet(1, 0, script["seed"], script["dt"])
        for o in script["ops"]:
            if o[0] == "create":
                probe.create(o[1], o[2])
        for k2 in want_adm:                       # the admitted requests before it, then this one
            probe.declare(*ops[k2][1:])
        cid = probe.declare(src, tgt, conn, syn, alpha)
        n = probe.call_count(cid, 0)
        cost = 14 * n + meta_bytes(op, script["dt"])
        if resident + cost <= budget:
            resident += cost
            want_adm.append(k)
            want_counts.append(n)
            want_status.append(0)
        else:
            want_status.append(-3)
    assert status == want_status and admitted == want_adm and counts == want_counts
    assert -3 in status and len(admitted) > 10
