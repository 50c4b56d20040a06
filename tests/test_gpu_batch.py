"""Batched uneven instances (persistent kernels in one captured HIP graph) and the q'-chunk
autotuner, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import configs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fp4():
    import paper_2104_04895_amd as m
    return m


@pytest.fixture(scope="module")
def instances():
    return [synth.small(),
            configs.wurtzite(grid=(2, 2, 2)),
            configs.layered(grid=(2, 2, 1)),
            synth.diamond_instance((3, 2, 2), configs.RC_SECOND, seed=12, T=(300.0, 700.0))]


def _ctx(fp4, inst, qchunk=0):
    c = fp4.Context(0)
    c.load_instance(inst, dq=oracle.default_dq(inst.cr.A, inst.grid))
    if qchunk:
        c.set_param(fp4.FP4_PARAM_QCHUNK, qchunk)
    return c


def _rel(a, b):
    den = np.maximum(np.abs(b), 1e-300)
    return np.max(np.where(b == 0, np.abs(a), np.abs(a - b) / den))


def test_batch_matches_single_contexts_and_replays(fp4, instances):
    """The graph-captured persistent batch gives the same counts and (to rounding) the same
    rates as each context alone; replays with eager work in between repeat bit for bit."""
    _say("case: batch vs single contexts")
    T = [300.0, 700.0]
    ctxs = [_ctx(fp4, inst, qchunk=q) for inst, q in zip(instances, (2, 3, 1, 4))]
    single = [c.compute_rates4(T, 1.0, 7, fp4.FP4_FP64) for c in ctxs]
    with fp4.Batch(0) as b:
        for c in ctxs:
            b.add(c)
        r1, c1 = b.compute(T, 1.0, 7, fp4.FP4_FP64)
        for i in range(len(ctxs)):
            assert np.array_equal(c1[i], single[i][2])
            assert _rel(r1[i], single[i][0]) <= 1e-13
        for rep in range(3):
            ctxs[0].compute_rates4([500.0], 1.0, 7, fp4.FP4_FP64)   # eager work between replays
            r2, c2 = b.compute(T, 1.0, 7, fp4.FP4_FP64)
            for i in range(len(ctxs)):
                assert np.array_equal(r2[i], r1[i]) and np.array_equal(c2[i], c1[i])
        t = b.last_timing()
        assert t["graph_builds"] == 1 and t["graph_launches"] == 4
        # new temperatures are read by the same graph at replay time
        r3, _ = b.compute([450.0, 900.0], 1.0, 7, fp4.FP4_FP64)
        assert b.last_timing()["graph_builds"] == 1
    for i, c in enumerate(ctxs):
        ref, _, _ = c.compute_rates4([450.0, 900.0], 1.0, 7, fp4.FP4_FP64)
        assert _rel(r3[i], ref) <= 1e-13
        c.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-4)])
def test_batch_against_oracle(fp4, instances, precision, tol):
    """Per-instance parity of the batched path with the FP64 oracle on sampled modes
    (4-atom instances: 12 branches, ~3900 quartets)."""
    _say("case: batch vs oracle", precision)
    T = [300.0, 700.0]
    ctxs = [_ctx(fp4, inst) for inst in instances]
    with fp4.Batch(0) as b:
        for c in ctxs:
            b.add(c)
        r, cnt = b.compute(T, 1.0, 7, precision)
    rng = np.random.default_rng(5)
    for i, inst in enumerate(instances):
        tg = rng.choice(np.arange(3, inst.nmodes), 3, replace=False)
        m = oracle.Model.from_instance(inst)
        r_o, _, c_o = oracle.rates4(m, T, 1.0, 7, oracle.default_dq(inst.cr.A, inst.grid), tg)
        assert np.array_equal(cnt[i][tg], c_o)
        err = _rel(r[i][:, tg], r_o)
        _say(inst.name, "max rel err", err)
        assert err <= tol
    for c in ctxs:
        c.close()


def test_autotune(fp4, instances):
    """The autotuner times every candidate chunk size, keeps the fastest in the context, and
    the rates do not depend on the choice beyond rounding."""
    _say("case: autotune")
    inst = instances[0]
    with _ctx(fp4, inst) as c:
        ref, _, cref = c.compute_rates4([300.0], 1.0, 7, fp4.FP4_FP64)
        best, times = fp4.autotune(c, [300.0], 1.0, 7, fp4.FP4_FP64, nsample=24)
        assert best in times and len(times) >= 2
        assert times[best] == min(times.values())
        r, _, cnt = c.compute_rates4([300.0], 1.0, 7, fp4.FP4_FP64)
    assert np.array_equal(cnt, cref)
    assert _rel(r, ref) <= 1e-13


def test_autotune_shapes(fp4, instances):
    """The work-shape autotuner tries the q'-chunks, then queue and list segments at the best
    chunk, keeps the fastest configuration in the context; any setting of the segments (here
    also the smallest, 64 and 64, which forces many phases and passes) gives the same counts
    and rates equal to rounding, and the oracle's rates within 1e-10."""
    _say("case: autotune shapes")
    inst = instances[0]
    m = oracle.Model.from_instance(inst)
    r_o, _, c_o = oracle.rates4(m, [300.0, 700.0], 1.0, 7, oracle.default_dq(inst.cr.A, inst.grid))
    with _ctx(fp4, inst) as c:
        best, tried = fp4.autotune_shapes(c, [300.0, 700.0], 1.0, 7, fp4.FP4_FP64, nsample=24)
        cfgs = [cfg for cfg, _ in tried]
        assert best in cfgs and len(cfgs) >= 4
        assert dict(tried)[best] == min(ms for _, ms in tried)
        assert len({(q, l) for _, q, l in cfgs}) >= 2
        r, _, cnt = c.compute_rates4([300.0, 700.0], 1.0, 7, fp4.FP4_FP64)
        c.set_param(fp4.FP4_PARAM_QSEG, 64)
        c.set_param(fp4.FP4_PARAM_LSEG, 64)
        r64, _, cnt64 = c.compute_rates4([300.0, 700.0], 1.0, 7, fp4.FP4_FP64)
        r32, _, cnt32 = c.compute_rates4([300.0, 700.0], 1.0, 7, fp4.FP4_FP32)
        with pytest.raises(fp4.Fp4Error):
            c.set_param(fp4.FP4_PARAM_QSEG, 100)
    assert np.array_equal(cnt, c_o) and np.array_equal(cnt64, c_o) and np.array_equal(cnt32, c_o)
    assert _rel(r, r_o) <= 1e-10 and _rel(r64, r_o) <= 1e-10
    assert _rel(r64, r) <= 1e-12
    assert _rel(r32, r_o) <= 1e-4
