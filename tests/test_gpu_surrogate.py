"""The learned surrogate end to end on the GPU: features (incl. the three-phonon rate),
training by the library's kernels, BF16 inference on a denser grid, flagging, exact
fallback and audit; checked against the exact kernel on every mode of the inference grid.

Shows the gain: the whole surrogate pass (features, inference, fallback and audit) takes
less time than the exact kernel on all modes, and the returned rates are within a stated
error of the exact ones (exact where the fallback or the audit recomputed them)."""
import json
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from synth.fc3 import random_fc3

pytestmark = pytest.mark.gpu

T_TRAIN = [100.0, 300.0, 600.0, 1200.0]
T_INF = [300.0, 700.0]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _load(fp4, grid, seed):
    inst = synth.diamond_instance(grid, synth.configs.RC_SECOND, seed=seed)
    fc3 = random_fc3(inst.cr, 3.0, np.random.default_rng(seed + 500))
    c = fp4.Context(0)
    c.load_instance(inst, dq=oracle.default_dq(inst.cr.A, inst.grid))
    c.load_fc3(fc3.atoms, fc3.cells, fc3.phi)
    return inst, c


@pytest.fixture(scope="module")
def trained():
    import paper_2104_04895_amd as fp4
    from paper_2104_04895_amd import surrogate as S
    _say("case: surrogate training on 6x6x6 draws")
    rng = np.random.default_rng(0)
    tr, ca = S.TrainSet(), S.TrainSet()
    for d in range(4):
        inst, c = _load(fp4, (6, 6, 6), 1000 + d)
        modes = rng.permutation(inst.nmodes)
        cut = inst.nmodes // 10
        X, y, _ = S.collect(c, inst.omega, T_TRAIN, 1.0, modes[cut:])
        tr.add(X, y)
        X, y, _ = S.collect(c, inst.omega, T_TRAIN, 1.0, modes[:cut])
        ca.add(X, y)
        c.close()
    sur = S.Surrogate(seed=1)
    X, y = tr.arrays()
    loss = sur.fit(X, y, epochs=40, batch=256, lr=1e-3)
    kappa = sur.calibrate(*ca.arrays())
    _say(f"rows {len(y)} loss {loss[0]:.3f} -> {loss[-1]:.3f} kappa {kappa:.2f}")
    yield fp4, S, sur
    sur.close()


def test_surrogate_gain_on_denser_grid(trained, tmp_path):
    fp4, S, sur = trained
    _say("case: surrogate inference on the 8x8x8 grid of a training draw")
    inst, c = _load(fp4, (8, 8, 8), 1000)
    rates, rep = S.infer(sur, c, inst.omega, T_INF, flag_sigma=0.15, audit_frac=0.05,
                         audit_seed=3)
    t0 = time.perf_counter()
    r_ex, _, _ = c.compute_rates4(T_INF, 1.0, 7, fp4.FP4_FP64, counts=False)
    t_exact = time.perf_counter() - t0
    c.close()
    act = np.flatnonzero(inst.omega.reshape(-1) > 0)
    recomputed = np.array(rep["audit_modes"] + rep["flagged_modes"], dtype=int)
    kept = np.setdiff1d(act, recomputed)
    # recomputed modes carry the exact kernel's rates (only the work split differs)
    np.testing.assert_allclose(rates[:, recomputed], r_ex[:, recomputed], rtol=1e-10)
    inactive = np.flatnonzero(inst.omega.reshape(-1) <= 0)
    assert np.all(rates[:, inactive] == 0)
    rel = np.abs(rates[:, kept] - r_ex[:, kept]) / r_ex[:, kept]
    true_med, true_p90 = float(np.median(rel)), float(np.quantile(rel, 0.9))
    rep_short = {k: v for k, v in rep.items() if k not in ("audit_modes", "flagged_modes")}
    rep_short["true_rel_err_kept"] = {"median": true_med, "p90": true_p90,
                                      "max": float(rel.max())}
    rep_short["exact_all_modes_seconds_measured"] = t_exact
    _say(json.dumps(rep_short))
    # the surrogate's error on the modes whose prediction is kept
    assert true_med < 0.10 and true_p90 < 0.30
    # the audit's estimate of it is consistent with the truth
    assert abs(rep["audit_rel_err"]["median"] - true_med) < 0.5 * true_med + 0.02
    # fewer than a quarter of the modes fall back, and the whole pass beats the exact kernel
    assert rep["fallback_frac"] < 0.25
    assert rep["seconds"]["total"] < t_exact
    # checkpoint round trip reproduces the predictions
    sur.save(str(tmp_path / "sur"))
    s2 = S.Surrogate.load(str(tmp_path / "sur"))
    X = np.random.default_rng(1).standard_normal((64, fp4.FP4_NFEAT)).astype(np.float32)
    a = sur.predict(X)
    b = s2.predict(X)
    s2.close()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_surrogate_flags_out_of_range(trained):
    fp4, S, sur = trained
    _say("case: surrogate range flag")
    X = np.tile(sur.shift, (3, 1)).astype(np.float32)
    X[1, 15] = sur.hi[15] + 5.0          # three-phonon rate far above anything trained on
    X[2, 2:14] = 0.0
    X[2, 13] = 1.0                       # branch 11: never seen for a 6-branch crystal
    assert list(sur.out_of_range(X)) == [False, True, True]
