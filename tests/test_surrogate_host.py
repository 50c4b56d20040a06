"""Host logic of the surrogate driver on the CPU, with stand-ins for the library calls:
flagging, the audit sample, replacement by exact rates, the error report and the chunked
exact calls.  (The network, the features and the exact kernel are tested on the GPU.)"""
import numpy as np
import pytest

from paper_2104_04895_amd import FP4_NFEAT
from paper_2104_04895_amd import surrogate as S


class FakeCtx:
    """Exact rate of mode m at temperature t: (m + 1) * (t + 1); features carry the mode id."""

    def __init__(self, nmodes):
        self.nmodes = nmodes
        self.calls = []

    def surrogate_features(self, T, sb, targets):
        X = np.zeros((len(T), len(targets), FP4_NFEAT), dtype=np.float32)
        X[:, :, 0] = np.asarray(targets)[None, :]
        return X, np.zeros((len(T), len(targets)))

    def compute_rates4(self, T, sb, mask, precision, targets, counts=False):
        targets = np.asarray(targets)
        self.calls.append(len(targets))
        r = (targets[None, :] + 1.0) * (np.arange(len(T))[:, None] + 1.0)
        return r, None, None


class FakeSur:
    """Predicts the exact rate times 1.1 (10% error); sigma large for modes divisible by 7;
    mode 5 is out of range."""

    def predict(self, X, bf16=True):
        m = X[:, 0].astype(np.int64)
        nT = len(X) // len(np.unique(m))
        t = np.repeat(np.arange(nT), len(X) // nT)
        mu = np.log(1.1 * (m + 1.0) * (t + 1.0))
        sig = np.where(m % 7 == 0, 1.0, 0.05)
        return mu, sig, 0.0

    def out_of_range(self, X):
        return X[:, 0] == 5


def test_infer_flags_audit_and_replacement():
    nm = 200
    omega = np.ones(nm)
    omega[:3] = 0.0                                   # inactive modes
    ctx, sur = FakeCtx(nm), FakeSur()
    T = [300.0, 700.0]
    rates, rep = S.infer(sur, ctx, omega, T, flag_sigma=0.2, audit_frac=0.05, audit_seed=1,
                         chunk=16)
    exact = (np.arange(nm)[None, :] + 1.0) * np.array([[1.0], [2.0]])
    active = np.arange(3, nm)
    flagged = np.array(rep["flagged_modes"])
    audited = np.array(rep["audit_modes"])
    assert set(flagged) == {m for m in active if m % 7 == 0 or m == 5}
    assert len(audited) == round(0.05 * len(active))
    assert not set(flagged) & set(audited)
    # recomputed modes carry exact rates, the others the prediction, inactive modes zero
    rec = np.concatenate([flagged, audited])
    np.testing.assert_allclose(rates[:, rec], exact[:, rec])
    kept = np.setdiff1d(active, rec)
    np.testing.assert_allclose(rates[:, kept], 1.1 * exact[:, kept])
    assert np.all(rates[:, :3] == 0.0)
    # the audit reports the 10% error of the kept predictions
    assert abs(rep["audit_rel_err"]["median"] - 0.1) < 1e-12
    assert rep["fallback_frac"] == (len(flagged) + len(audited)) / len(active)
    # exact work went out in chunks of at most 16 modes
    assert max(ctx.calls) <= 16 and sum(ctx.calls) == len(rec)


def test_exact_chunked_reports_progress():
    ctx = FakeCtx(100)
    seen = []
    r, _, done = S.exact_chunked(ctx, [300.0], 1.0, np.arange(37), chunk=10,
                                 progress=lambda w, d, t: seen.append((d, t)))
    assert seen == [(10, 37), (20, 37), (30, 37), (37, 37)]
    assert done.all()
    np.testing.assert_allclose(r[0], np.arange(37) + 1.0)


def test_exact_chunked_resumes_from_checkpoint(tmp_path):
    """A pass stopped by its deadline after the first chunk leaves that chunk on disk; the
    second pass reads it back and computes only the rest, with the same result."""
    import time
    ctx = FakeCtx(100)
    r1, _, done1 = S.exact_chunked(ctx, [300.0], 1.0, np.arange(37), chunk=10, what="flagged",
                                   ckpt=str(tmp_path), deadline=time.perf_counter() - 1.0)
    assert not done1.any() and sum(ctx.calls) == 0          # past the deadline: nothing starts
    calls = []
    ctx2 = FakeCtx(100)
    ctx2.calls = calls
    S.exact_chunked(ctx2, [300.0], 1.0, np.arange(37)[:10], chunk=10, what="flagged",
                    ckpt=str(tmp_path))                          # writes chunk 0 (targets 0..9)
    assert calls == [10]
    ctx3 = FakeCtx(100)
    r3, t3, done3 = S.exact_chunked(ctx3, [300.0], 1.0, np.arange(37), chunk=10, what="flagged",
                                    ckpt=str(tmp_path))
    assert done3.all() and ctx3.calls == [10, 10, 7]          # chunk 0 read back
    np.testing.assert_allclose(r3[0], np.arange(37) + 1.0)
    # the seconds of every chunk are on disk, and a pass that reads them all back reports
    # their sum as its exact time
    secs = sum(float(np.load(tmp_path / f"flagged_{a:08d}_{n}_seconds.npy")[0])
               for a, n in ((0, 10), (10, 10), (20, 10), (30, 7)))
    ctx5 = FakeCtx(100)
    _, t5, done5 = S.exact_chunked(ctx5, [300.0], 1.0, np.arange(37), chunk=10, what="flagged",
                                   ckpt=str(tmp_path))
    assert done5.all() and ctx5.calls == [] and t5 == pytest.approx(secs) and t5 >= t3
    # a chunk file whose target list differs is recomputed, not trusted
    ctx4 = FakeCtx(100)
    S.exact_chunked(ctx4, [300.0], 1.0, np.arange(1, 38), chunk=10, what="flagged",
                    ckpt=str(tmp_path))
    assert ctx4.calls == [10, 10, 10, 7]
