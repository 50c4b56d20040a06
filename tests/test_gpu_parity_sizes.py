"""GPU parity at the benchmarked sizes, against the FP64 oracle's values.

The oracle is too slow to run on complete modes of these grids inside the test (minutes to
tens of minutes per mode), so its values were written by `tests/golden/make_oracle_values.py`,
which calls only `oracle/`.  Every stored record carries a fingerprint of the inputs it was
computed from; the test regenerates the seeded workload, and uses the stored values only if
its fingerprint matches.  Otherwise (a different BLAS could change the last bits of the
eigenvectors) the counts are recomputed by the oracle live, and the stored rates are skipped
with that reason.

Bar: kept-process counts bit-exact; FP64 rates within 1e-10 relative; FP32 within 1e-4.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import configs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_oracle_values import fingerprint  # noqa: E402

RTOL64 = 1e-10
RTOL32 = 1e-4
GOLDEN = os.path.join(HERE, "golden", "oracle_values.json")


def _say(*a):
    print(*a, flush=True)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    den = np.maximum(np.abs(b), 1e-300)
    return float(np.max(np.where(b == 0, np.abs(a), np.abs(a - b) / den)))


@pytest.fixture(scope="module")
def fp4():
    import paper_2104_04895_amd as m
    return m


def _stored(name, inst):
    """The stored oracle record of this workload, or None when the inputs differ."""
    with open(GOLDEN) as f:
        data = json.load(f)
    rec = data[name]
    fp = fingerprint(inst)
    same = fp == rec["fingerprint"]
    _say(f"{name}: input fingerprint {'matches' if same else 'DIFFERS from'} the stored oracle run")
    return rec if same else None


def _live_counts(inst, case):
    m = oracle.Model.from_instance(inst)
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    _, _, c = oracle.rates4(m, case["T"], case["scalebroad"], case["mask"], dq,
                            np.array(case["targets"], np.int32), want_rates=False)
    return c


def _ctx(fp4, inst):
    c = fp4.Context(0)
    c.load_instance(inst, dq=oracle.default_dq(inst.cr.A, inst.grid))
    return c


def test_medium_complete_modes(fp4):
    """8x8x8 second-shell workload, T = 300/1000 K, full grid in the benchmark's launch
    configuration: complete rates (all channels) of 4 modes, among them the lowest-frequency
    non-Gamma acoustic mode (the binding case for FP32 cancellation), FP64 within 1e-10 and
    FP32 within 1e-4; counts exact."""
    inst = synth.medium()
    with open(GOLDEN) as f:
        case = json.load(f)["medium-8x8x8"]["cases"]["full"]
    rec = _stored("medium-8x8x8", inst)
    tg = np.array(case["targets"])
    _say("case: medium 8x8x8, complete rates of modes", tg.tolist())
    with _ctx(fp4, inst) as c:
        r, rch, cnt = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64, by_channel=True)
        r32, _, cnt32 = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP32)
    ref_c = np.array(case["counts"]) if rec else _live_counts(inst, case)
    assert np.array_equal(cnt[tg], ref_c) and np.array_equal(cnt32[tg], ref_c)
    if rec is None:
        pytest.skip("inputs differ from the stored oracle run: counts checked live, rates skipped")
    ro, rcho = np.array(case["rates"]), np.array(case["rates_by_channel"])
    e64, e32 = _rel(r[:, tg], ro), _rel(r32[:, tg], ro)
    _say(f"  max rel err FP64 {e64:.2e}, FP32 {e32:.2e}")
    assert e64 <= RTOL64 and _rel(rch[:, :, tg], rcho) <= RTOL64
    assert e32 <= RTOL32


def test_large_sampled_modes(fp4):
    """16x16x16 workload (the paper's BAs grid): counts of 8 sampled modes at scalebroad 1 and
    0.1 bit-exact; recombination and splitting rates of 3 of them at scalebroad 1; the complete
    rate of one mode at scalebroad 0.1 (the paper's setting), FP64 1e-10 and FP32 1e-4."""
    inst = synth.large()
    with open(GOLDEN) as f:
        cases = json.load(f)["large-16x16x16"]["cases"]
    rec = _stored("large-16x16x16", inst)
    with _ctx(fp4, inst) as c:
        for key in ("counts", "counts_sb01"):
            case = cases[key]
            tg = np.array(case["targets"], np.int32)
            _say(f"case: large 16x16x16 counts sb {case['scalebroad']}", tg.tolist())
            _, _, cnt = c.compute_rates4(case["T"], case["scalebroad"], 7, fp4.FP4_FP64, tg)
            ref_c = np.array(case["counts"]) if rec else _live_counts(inst, case)
            assert np.array_equal(cnt, ref_c)
        if rec is None:
            pytest.skip("inputs differ from the stored oracle run: counts checked live, rates skipped")
        for key in ("pp_mm", "full_sb01"):
            case = cases[key]
            tg = np.array(case["targets"], np.int32)
            _say(f"case: large 16x16x16 {key}", tg.tolist())
            r, rch, cnt = c.compute_rates4(case["T"], case["scalebroad"], case["mask"],
                                           fp4.FP4_FP64, tg, by_channel=True)
            r32, _, cnt32 = c.compute_rates4(case["T"], case["scalebroad"], case["mask"],
                                             fp4.FP4_FP32, tg)
            assert np.array_equal(cnt, np.array(case["counts"]))
            assert np.array_equal(cnt32, cnt)
            ro = np.array(case["rates"])
            e64, e32 = _rel(r, ro), _rel(r32, ro)
            _say(f"  max rel err FP64 {e64:.2e}, FP32 {e32:.2e}")
            assert e64 <= RTOL64 and _rel(rch, np.array(case["rates_by_channel"])) <= RTOL64
            assert e32 <= RTOL32


def test_batched_instances_configured_sizes(fp4):
    """The three instances of the batched workload at their configured grids (10x10x10 with 6
    branches, 8x8x6 and 6x6x6 with 12) in one persistent graph-captured launch with the FP32
    contraction, T = 300/700 K: counts of 8 sampled modes of each bit-exact; the complete rate
    of one mode of each from the batch (FP32, 1e-4) and from a single FP64 call (1e-10)."""
    names = ["cubic-10x10x10", "wurtzite-8x8x6", "layered-6x6x6"]
    insts = [configs.cubic10(), configs.wurtzite(), configs.layered()]
    with open(GOLDEN) as f:
        data = json.load(f)
    recs = [_stored(n, i) for n, i in zip(names, insts)]
    T = insts[0].T
    ctxs = [_ctx(fp4, i) for i in insts]
    try:
        _say("case: batched workload, one graph, FP32")
        with fp4.Batch(0) as b:
            for c in ctxs:
                b.add(c)
            rb, cb = b.compute(T, 1.0, 7, fp4.FP4_FP32)
        missing = []
        for k, (name, inst, rec, c) in enumerate(zip(names, insts, recs, ctxs)):
            cases = data[name]["cases"]
            tg = np.array(cases["counts"]["targets"], np.int32)
            ref_c = np.array(cases["counts"]["counts"]) if rec else _live_counts(inst, cases["counts"])
            assert np.array_equal(cb[k][tg], ref_c), name
            if rec is None:
                missing.append(name)
                continue
            one = np.array(cases["full"]["targets"], np.int32)
            r64, _, c64 = c.compute_rates4(T, 1.0, 7, fp4.FP4_FP64, one)
            ro = np.array(cases["full"]["rates"])
            assert np.array_equal(c64, np.array(cases["full"]["counts"])), name
            e64, e32 = _rel(r64, ro), _rel(rb[k][:, one], ro)
            _say(f"  {name} mode {int(one[0])}: FP64 {e64:.2e}, FP32 batch {e32:.2e}")
            assert e64 <= RTOL64, name
            assert e32 <= RTOL32, name
        if missing:
            pytest.skip(f"inputs differ from the stored oracle run for {missing}: counts checked live, rates skipped")
    finally:
        for c in ctxs:
            c.close()
