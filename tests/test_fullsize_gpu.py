"""Parity at the benchmark's full sizes, element by element, in the launch
configuration the bench uses.

The oracle's whole result at these sizes is reassembled by the full-size
harness (tests/fullsize_oracle.py: the plain C oracle in 16 worker processes,
pinned against the oracle's whole run by tests/test_fullsize_harness.py):

  * column8 (4.1e8 connections), multi-area point-to-point share (6.4e8) and
    balanced collective share (2.25e9): every sorted connection (source',
    target, delay; weight within 2 ulp), every row of the first-index array,
    the whole image map (R, L, img_base), the point-to-point send lists S and
    T/P, and the collective H, I, G, Q -- all equal the oracle's;
  * the served stream (10,000 requests, 64 GiB budget): every admission
    decision and every admitted request's connection count against the
    oracle's admission (its counts under the documented resident cost), the
    whole first-index array, and the complete rows of 2,000 random sources
    and of the 50 largest rows.
"""
import os
import shutil
import time

import numpy as np
import pytest

import oracle
import paper_2512_09502_amd as snnc
from fullsize_oracle import FullSizeOracle, dump_library_arrays, served_admission
from gpu_util import log
from paper_2512_09502_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

WORKERS = 16


def _torch():
    import torch
    torch.cuda.set_device(0)
    return torch


@pytest.fixture
def scratch(tmp_path):
    base = "/dev/shm" if os.path.isdir("/dev/shm") else str(tmp_path)
    d = os.path.join(base, f"snnc_fullsize_{os.getpid()}_{time.monotonic_ns()}")
    os.makedirs(d)
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _connect_ops(script):
    return [op for op in script["ops"] if op[0] == "connect"]


def _whole(script, P_local, scratch, maps=(), extra=()):
    """Build on the GPU, dump the prepared arrays, and compare everything
    with the oracle's reassembled result."""
    _torch()
    t0 = time.time()
    net = snnc.run_script(script, P_local)
    names = ["src", "tgt", "delay", "weight", "row_ptr"]
    gpu_dir = os.path.join(scratch, "gpu")
    dump_library_arrays(net, gpu_dir, names)
    small = {k: net.array(k) for k in list(maps) + list(extra)}
    n = net.count("src")
    net.close()
    log(f"{script['name']} host {P_local}: {n} connections built and copied out in {time.time() - t0:.1f} s")
    h = FullSizeOracle(script, P_local, _connect_ops(script), os.path.join(scratch, "oracle"), workers=WORKERS,
                       log=log)
    try:
        t0 = time.time()
        h.generate()
        assert h.n_generated == n, f"oracle generates {h.n_generated}, library holds {n}"
        log(f"oracle phase A + image map: {time.time() - t0:.1f} s")
        t0 = time.time()
        m, errors = h.compare(gpu_dir)
        log(f"oracle phase B: {m} connections compared in {time.time() - t0:.1f} s")
        assert errors == [], errors[:5]
        assert m == n
        want = {}
        if "r_off" in maps:
            want.update(h.image_map())
        if "s_off" in extra:
            want.update(h.send_lists())
        if "h_off" in extra:
            want.update(h.collective())
        for k, got in small.items():
            np.testing.assert_array_equal(got, want[k].astype(got.dtype), err_msg=k)
        log(f"{script['name']}: every connection, row, map and list equal the oracle's "
            f"({', '.join(sorted(small)) or 'no maps'})")
    finally:
        h.close()


def test_column8_full_size(scratch):
    _whole(W.column8(), 0, scratch)


def test_multiarea_p2p_full_size(scratch):
    _whole(W.multiarea_p2p(), 0, scratch, maps=("r_off", "r_val", "l_val", "img_base"),
           extra=("s_off", "s_val", "tp_ptr", "t_val", "p_val"))


def test_collective_full_size(scratch):
    _whole(W.balanced_collective(), 0, scratch, maps=("r_off", "r_val", "l_val", "img_base"),
           extra=("groups", "h_off", "h_val", "i_val", "gq_ptr", "g_val", "q_val"))


# ---------------------------------------------------------------- served stream
def test_served_full_size(scratch):
    torch = _torch()
    script = W.served_requests()
    budget = 64 << 30
    ops = _connect_ops(script)
    t0 = time.time()
    status, admitted, count_of = served_admission(script, budget, workers=WORKERS)
    log(f"served: oracle admission of {len(ops)} requests in {time.time() - t0:.1f} s: "
        f"{len(admitted)} admitted, {sum(count_of)} connections")
    # the library, built as the bench builds it (batches of 256 through snnc_submit_many)
    t0 = time.time()
    net = snnc.Network(1, 0, script["seed"], script["dt"])
    net.set_resident_budget(budget)
    for op in script["ops"]:
        if op[0] == "create":
            net.create(op[1], op[2])
    batch = snnc.RequestBatch([op[1:] for op in ops])
    got_status = []
    for k0 in range(0, len(ops), 256):
        got_status.extend(st for st, _ in net.submit_batch(batch, k0, k0 + 256))
        net.flush()
    net.sync()
    assert got_status == status, [(k, a, b) for k, (a, b) in enumerate(zip(got_status, status)) if a != b][:10]
    off = net.array("call_off").astype(np.int64)
    np.testing.assert_array_equal(np.diff(off), np.array(count_of, np.int64))
    net.prepare()
    gpu_dir = os.path.join(scratch, "gpu")
    dump_library_arrays(net, gpu_dir)
    n = net.count("src")
    net.close()
    del torch
    log(f"served: library admission and per-request counts equal the oracle's; {n} connections built and "
        f"copied out in {time.time() - t0:.1f} s")
    rp = np.load(os.path.join(gpu_dir, "row_ptr.npy"), mmap_mode="r")
    M = rp.size - 1
    rng = np.random.default_rng(5)
    select = np.zeros(M, bool)
    select[rng.choice(M, size=2000, replace=False)] = True
    select[np.argsort(np.diff(np.asarray(rp, dtype=np.int64)))[-50:]] = True     # the largest rows
    kept = dict(script)
    calls = [ops[k] for k in admitted]
    h = FullSizeOracle(kept, 0, calls, os.path.join(scratch, "oracle"), workers=WORKERS, select=select,
                       row_counts=True, log=log)
    try:
        t0 = time.time()
        h.generate()
        assert h.n_generated == n
        np.testing.assert_array_equal(np.diff(np.asarray(rp, dtype=np.int64)), h.rows)
        m, errors = h.compare(gpu_dir)
        assert errors == [], errors[:5]
        log(f"served: whole first-index array and {int(select.sum())} complete rows ({m} connections) equal the "
            f"oracle's ({time.time() - t0:.1f} s)")
    finally:
        h.close()


def test_indegree_x10_full_size(scratch):
    # the in-degree sweep's largest scale: K = 90,000 + 22,500 per target, 1.6e4 + 4e3 sources per host
    _whole(W.balanced_indegree(10), 0, scratch, maps=("r_off", "r_val", "l_val", "img_base"),
           extra=("groups", "h_off", "h_val", "i_val", "gq_ptr", "g_val", "q_val"))
