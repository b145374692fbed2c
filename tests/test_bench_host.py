"""Host logic of bench.py (no GPU): the single-GPU guard, the reserve hint a
workload states for the host, the phase grouping of kernel times, and the
traffic table's source-hash check."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2512_09502_amd import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_reserve_hint_per_host():
    s = W.multiarea_p2p(P=4, n_e=100, n_i=25, k_e=10, k_i=3, k_remote_max=5, seed=3)
    kr = s["info"]["k_remote"]
    for tau in range(4):
        remote = sum(kr[sigma][tau] for sigma in range(4) if sigma != tau)
        assert bench.expected_conns(s, tau) == 125 * (13 + remote)
    assert bench.expected_conns(W.column8(scale=0.01)) == W.column8(scale=0.01)["info"]["conns"]


def test_phase_grouping():
    kernels = {"gen_total": (4, 4.0), "prep_keys": (1, 2.0), "prep_number": (1, 1.5), "sort_pass": (3, 9.0),
               "sort_pass_final": (1, 3.0), "prep_csr": (1, 0.5), "prep_mark": (2, 1.0), "scan": (5, 0.25),
               "gen_total_sort_pass": (6, 2.0), "gen_total_sort_hist_scan": (2, 0.5)}
    out = bench.phase_times(kernels, {"ms_connect": 5.0, "ms_prepare": 15.0})
    # the radix sorts that generation runs count as generation, not as the sort+index phase
    assert out["generation"] == 6.5 and out["keys_unique_remap"] == 3.5 and out["sort"] == 12.0
    assert out["csr"] == 0.5 and out["send_lists"] == 1.0 and out["other"] == 0.25
    assert out["connect_events_ms"] == 5.0 and out["prepare_events_ms"] == 15.0


def test_traffic_table_follows_the_sort_source():
    # the committed counters are used only while the kernel source they were taken on is unchanged
    import hashlib
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    e = next(x for x in t["entries"] if x["kernel"] == "sort_pass")
    n = 408483244
    got = bench.measured_traffic("sort_pass", n, e["workload"])
    sha = hashlib.sha1(open(os.path.join(ROOT, e["source"]), "rb").read()).hexdigest()
    if sha == e["sha1"]:
        assert got == pytest.approx(n * (e["read_bytes_per_elem"] + e["write_bytes_per_elem"]), rel=1e-6)
    else:
        assert got is None
    assert bench.measured_traffic("sort_pass", n, "some_other_workload") is None


def test_sort_roofline_figures():
    # dominant pass at 28 B per connection over its average launch time; the
    # phase figure sums every Prepare kernel of the bracketed build
    n = 10**9
    timed = {"sort_pass": (8, 80.0), "sort_pass_final": (2, 24.0), "gen_fused": (5, 400.0)}
    breakdown = {"prep_keys": (1, 5.0), "sort_pass": (4, 40.0), "sort_pass_final": (1, 12.0), "prep_csr": (1, 1.0),
                 "gen_fused": (3, 100.0)}
    r = bench.sort_roofline(timed, breakdown, n, {"row_ptr": 1001}, "no_such_workload")
    assert r["kernel"] == "sort_pass" and r["avg_launch_ms"] == 10.0
    assert r["achieved"] == pytest.approx(28 * n / 10e-3 / 1e9, rel=1e-6)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["traffic"] is None
    ph = r["phase_sort_index"]
    assert ph["kernels_ms"] == 58.0
    assert ph["algorithmic_bytes"] == 28 * n + 8 * 1001
    assert bench.index_bytes({"row_ptr": 3, "r_val": 2, "i_val": 5, "tp_ptr": 4}) == 8 * 3 + 4 * 7 + 8 * 4
