"""Helpers for the GPU parity tests: build both sides from one script and
compare every array (integers bit-exact, fp32 weights within 2 ulp)."""
import sys

import numpy as np

import oracle
import paper_2512_09502_amd as snnc

GEN_ARRAYS = ["gen_src", "gen_tgt", "gen_delay", "gen_weight"]
PREP_ARRAYS = ["src", "tgt", "delay", "weight", "row_ptr", "r_off", "r_val", "l_val", "img_base", "s_off", "s_val",
               "tp_ptr", "t_val", "p_val", "groups", "h_off", "h_val", "i_val", "gq_ptr", "g_val", "q_val"]
LEVEL_ARRAYS = ["img_first", "img_count"]      # exist at some GPU memory levels only
WEIGHT_ULP = 2


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def ulp_diff(a: np.ndarray, b: np.ndarray) -> int:
    """max distance in fp32 units in the last place (same-sign values)"""
    if a.size == 0:
        return 0
    ia = a.view(np.int32).astype(np.int64)
    ib = b.view(np.int32).astype(np.int64)
    # map to a monotone integer line so that -0/+0 and sign changes count correctly
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return int(np.abs(ia - ib).max())


def compare(name: str, got: np.ndarray, ref: np.ndarray, what: str = ""):
    assert got.shape == ref.shape, f"{what} {name}: shape {got.shape} != oracle {ref.shape}"
    if name.endswith("weight"):
        d = ulp_diff(got, ref)
        assert d <= WEIGHT_ULP, f"{what} {name}: {d} ulp from the oracle"
    else:
        if not np.array_equal(got, ref.astype(got.dtype)):
            bad = np.nonzero(got != ref.astype(got.dtype))[0]
            raise AssertionError(f"{what} {name}: {bad.size} of {got.size} differ, first at {bad[0]}: "
                                 f"{got[bad[0]]} vs oracle {ref[bad[0]]}")


def build_pair(script, P_local, skip_invalid=True):
    """GPU network (prepared) and oracle network for one host; the
    generation-order arrays are captured before prepare."""
    log(f"case {script.get('name')} P={script['P']} P_local={P_local}")
    net = snnc.run_script(script, P_local, prepare=False, skip_invalid=skip_invalid)
    gen = {k: net.array(k) for k in GEN_ARRAYS}
    gen["call_off"] = net.array("call_off")
    net.prepare()
    ref = oracle.run_script(script, P_local, skip_invalid=skip_invalid)
    assert [k for k, _ in net.rejected] == [k for k, _ in ref.rejected]
    assert [c for _, c in net.rejected] == [c for _, c in ref.rejected]
    return net, gen, ref


def compare_all(script, P_local, skip_invalid=True):
    net, gen, ref = build_pair(script, P_local, skip_invalid)
    what = f"{script.get('name')}[P_local={P_local}]"
    for k in GEN_ARRAYS:
        compare(k, gen[k], ref.array(k), what)
    compare("call_off", gen["call_off"], ref.array("call_off"), what)
    for k in PREP_ARRAYS:
        compare(k, net.array(k), ref.array(k), what)
    for k in LEVEL_ARRAYS:
        try:
            want = ref.array(k)
        except oracle.OracleError:
            with np.testing.assert_raises(snnc.SnncError):
                net.array(k)
            continue
        compare(k, net.array(k), want, what)
    n = net.count("src")
    net.close()
    return n
