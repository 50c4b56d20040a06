"""Learned surrogate of the per-mode four-phonon rate, with exact fallback and audit.

The network (``Mlp``: `depth` linear layers of `width`, SiLU, a mean head and a log-sigma
head, Gaussian negative log-likelihood) is trained by the library's own FP32 kernels on
exact rates that the four-phonon kernel computes for a sampled subset of modes, and is
evaluated with BF16 weights and activations.  Input rows come from
``fp4_surrogate_features`` (frequency, speed, branch, occupation, three-phonon rate of
Eq. 3phgamma, temperature and the mode's fourth-order coupling strength), target = ln of the
rate of Eq. 4phgamma.

Inference on a new grid: predict every active mode, flag a mode when its predicted standard
deviation of ln(rate) exceeds ``flag_sigma`` at any temperature or when a feature lies
outside the range seen in training; compute flagged modes and a random audit sample of the
rest with the exact kernel, replace their predictions, and report the audit's measured
error (the audit is drawn from the modes that keep their prediction, so its error is an
unbiased estimate of the error of what is returned).

This module only orchestrates calls to the library (features, exact rates, training,
inference); the arithmetic runs in its kernels.  Python here standardises arrays, picks
samples and keeps statistics.
"""
from __future__ import annotations

import json
import time
from dataclasses import dataclass, field

import numpy as np

from . import FP4_FP64, FP4_NFEAT, Context, Mlp

CONTINUOUS = [0, 1, 14, 15, 16, 17]   # feature columns checked against the training range
ONEHOT = list(range(2, 14))


@dataclass
class TrainSet:
    X: list = field(default_factory=list)   # raw feature rows (float32, FP4_NFEAT)
    y: list = field(default_factory=list)   # ln rate

    def add(self, X, y):
        self.X.append(np.asarray(X, np.float32))
        self.y.append(np.asarray(y, np.float32))

    def arrays(self):
        return np.concatenate(self.X), np.concatenate(self.y)


def collect(ctx: Context, omega, T, scalebroad, targets, precision=FP4_FP64):
    """Exact rates and feature rows of `targets` (active modes with a non-zero rate only).
    Returns (X [n][FP4_NFEAT], y [n], seconds spent in the exact kernel)."""
    targets = np.asarray(targets, dtype=np.int32)
    targets = targets[np.asarray(omega).reshape(-1)[targets] > 0]
    X, _ = ctx.surrogate_features(T, scalebroad, targets)
    t0 = time.perf_counter()
    r4, _, _ = ctx.compute_rates4(T, scalebroad, 7, precision, targets, counts=False)
    t_exact = time.perf_counter() - t0
    keep = r4 > 0                                  # [nT][nt]
    return X[keep], np.log(r4[keep]).astype(np.float32), t_exact


class Surrogate:
    def __init__(self, width=128, depth=5, seed=0, device=0):
        self.width, self.depth, self.seed, self.device = width, depth, seed, device
        self.net = Mlp(device, FP4_NFEAT, width, depth, seed)
        self.shift = self.scale = None
        self.y_mean = self.y_std = None
        self.lo = self.hi = None
        self.seen_branch = None
        self.loss = None
        self.kappa = 1.0

    # ------------------------------------------------------------------ training
    def fit(self, X, y, epochs=60, batch=256, lr=1e-3, seed=0):
        X = np.asarray(X, np.float32)
        y = np.asarray(y, np.float32)
        mean = X.mean(axis=0)
        std = X.std(axis=0)
        self.shift = mean.astype(np.float32)
        self.scale = np.where(std > 1e-6, 1.0 / np.maximum(std, 1e-6), 1.0).astype(np.float32)
        self.y_mean = float(y.mean())
        self.y_std = float(max(y.std(), 1e-6))
        span = X.max(axis=0) - X.min(axis=0)
        self.lo = X.min(axis=0) - 0.02 * span
        self.hi = X.max(axis=0) + 0.02 * span
        self.seen_branch = X[:, ONEHOT].max(axis=0) > 0.5
        Xs = ((X - self.shift) * self.scale).astype(np.float32)
        ys = ((y - self.y_mean) / self.y_std).astype(np.float32)
        self.loss = self.net.train(Xs, ys, epochs=epochs, batch=batch, lr=lr, seed=seed)
        return self.loss

    def calibrate(self, X, y, quantile=0.9):
        """Rescale the predicted standard deviation with rows held out of training, so that
        the `quantile` of |y - mu| / sigma matches that of a standard normal (the log-sigma
        head is fitted in-sample and is over-confident on unseen rows)."""
        self.kappa = 1.0
        mu, sig, _ = self.predict(X)
        z = np.abs(np.asarray(y, np.float64) - mu) / sig
        gauss = {0.5: 0.6745, 0.8: 1.2816, 0.9: 1.6449, 0.95: 1.96}[quantile]
        self.kappa = float(max(np.quantile(z, quantile) / gauss, 1e-3))
        return self.kappa

    # ------------------------------------------------------------------ inference
    def predict(self, Xraw, bf16=True):
        """ln-rate mean and (calibrated) standard deviation for raw feature rows, and the
        device time of the forward pass in ms."""
        Xs = ((np.asarray(Xraw, np.float32) - self.shift) * self.scale).astype(np.float32)
        out, ms = self.net.predict(Xs, bf16=bf16)
        mu = out[:, 0].astype(np.float64) * self.y_std + self.y_mean
        sig = np.exp(out[:, 1].astype(np.float64)) * self.y_std * self.kappa
        return mu, sig, ms

    def out_of_range(self, Xraw):
        X = np.asarray(Xraw)
        bad = np.any((X[:, CONTINUOUS] < self.lo[CONTINUOUS]) | (X[:, CONTINUOUS] > self.hi[CONTINUOUS]), axis=1)
        unseen = np.any((X[:, ONEHOT] > 0.5) & ~self.seen_branch[None, :], axis=1)
        return bad | unseen

    # ------------------------------------------------------------------ checkpoint
    def save(self, prefix):
        """Weights as a float32 .npy (no pickle) and the standardisation as JSON."""
        np.save(prefix + ".npy", self.net.get_params())
        meta = {"width": self.width, "depth": self.depth, "shift": self.shift.tolist(),
                "scale": self.scale.tolist(), "y_mean": self.y_mean, "y_std": self.y_std,
                "lo": self.lo.tolist(), "hi": self.hi.tolist(),
                "seen_branch": self.seen_branch.tolist(), "kappa": self.kappa}
        with open(prefix + ".json", "w") as f:
            json.dump(meta, f)

    @classmethod
    def load(cls, prefix, device=0):
        with open(prefix + ".json") as f:
            meta = json.load(f)
        s = cls(meta["width"], meta["depth"], 0, device)
        s.net.set_params(np.load(prefix + ".npy", allow_pickle=False))
        s.shift = np.asarray(meta["shift"], np.float32)
        s.scale = np.asarray(meta["scale"], np.float32)
        s.y_mean, s.y_std = meta["y_mean"], meta["y_std"]
        s.lo = np.asarray(meta["lo"], np.float32)
        s.hi = np.asarray(meta["hi"], np.float32)
        s.seen_branch = np.asarray(meta["seen_branch"], bool)
        s.kappa = float(meta["kappa"])
        return s

    def close(self):
        self.net.close()


def exact_chunked(ctx: Context, T, scalebroad, targets, precision=FP4_FP64, chunk=0,
                  progress=None, what="exact", ckpt=None, deadline=None):
    """Exact rates of `targets` in calls of at most `chunk` modes (0: one call), reporting
    each finished call to `progress(what, done, total)`.

    With `ckpt` (a directory) every finished chunk is written there as
    `<what>_<first>_<n>.npy` (float64 [nT][n], no pickle) together with its target list and
    the seconds its exact call took, and chunks already present with the same targets are
    read back instead of recomputed, so an interrupted pass resumes where it stopped.  With
    `deadline` (a time.perf_counter() value) no new chunk starts after it.

    Returns (rates [nT][nt], seconds spent in the exact kernel, done [nt] bool); the seconds
    include those recorded with chunks read back (a chunk without a record counts zero)."""
    import os
    targets = np.asarray(targets, dtype=np.int32)
    nT = len(np.atleast_1d(T))
    out = np.zeros((nT, targets.size))
    done = np.zeros(targets.size, dtype=bool)
    step = targets.size if chunk <= 0 else chunk
    t_exact = 0.0
    for a in range(0, targets.size, max(step, 1)):
        tg = targets[a:a + step]
        path = os.path.join(ckpt, f"{what}_{a:08d}_{tg.size}.npy") if ckpt else None
        if path and os.path.exists(path) and os.path.exists(path[:-4] + "_targets.npy"):
            r = np.load(path, allow_pickle=False)
            same = np.array_equal(np.load(path[:-4] + "_targets.npy", allow_pickle=False), tg)
            if same and r.shape == (nT, tg.size):
                out[:, a:a + step] = r
                done[a:a + step] = True
                sec = path[:-4] + "_seconds.npy"
                if os.path.exists(sec):
                    t_exact += float(np.load(sec, allow_pickle=False).reshape(-1)[0])
                continue
        if deadline is not None and time.perf_counter() > deadline:
            continue
        t0 = time.perf_counter()
        r, _, _ = ctx.compute_rates4(T, scalebroad, 7, precision, tg, counts=False)
        dt = time.perf_counter() - t0
        t_exact += dt
        out[:, a:a + step] = r
        done[a:a + step] = True
        if path:
            np.save(path[:-4] + "_targets.npy", tg)
            np.save(path[:-4] + "_seconds.npy", np.array([dt]))
            np.save(path, r)
        if progress:
            progress(what, min(a + step, targets.size), targets.size)
    return out, t_exact, done


def infer(sur: Surrogate, ctx: Context, omega, T, scalebroad=1.0, flag_sigma=0.2,
          audit_frac=0.02, audit_seed=0, precision=FP4_FP64, bf16=True, chunk=0,
          progress=None, ckpt=None, max_exact_seconds=None):
    """Rates of every mode of the context's grid: surrogate predictions, with flagged modes
    and a random audit sample of the others recomputed by the exact kernel (in calls of at
    most `chunk` modes, each reported to `progress`).

    `ckpt` (a directory) keeps every finished exact chunk, so a pass cut short resumes
    where it stopped (see exact_chunked); `max_exact_seconds` stops starting new exact chunks
    after that much wall time, and the report's "complete" is then False.  An audited mode
    whose exact rate is zero (no kept process) while the prediction is positive counts as a
    miss: it is reported apart ("audit_zero_rate") and in the within-10% fraction.

    Returns (rates [nT][nq*nb], report dict)."""
    T = np.atleast_1d(np.asarray(T, np.float64))
    nT = len(T)
    omega = np.asarray(omega).reshape(-1)
    nmodes = omega.size
    active = np.flatnonzero(omega > 0).astype(np.int32)
    rep = {"modes": int(nmodes), "active": int(active.size), "T": T.tolist()}

    t0 = time.perf_counter()
    X, r3 = ctx.surrogate_features(T, scalebroad, active)          # [nT][na][F]
    t_feat = time.perf_counter() - t0
    t0 = time.perf_counter()
    mu, sig, ms_net = sur.predict(X.reshape(-1, FP4_NFEAT), bf16=bf16)
    t_pred = time.perf_counter() - t0
    mu = mu.reshape(nT, -1)
    sig = sig.reshape(nT, -1)
    oor = sur.out_of_range(X.reshape(-1, FP4_NFEAT)).reshape(nT, -1)
    flagged = np.any(sig > flag_sigma, axis=0) | np.any(oor, axis=0)
    rest = np.flatnonzero(~flagged)
    rng = np.random.default_rng(audit_seed)
    n_audit = int(round(audit_frac * active.size))
    n_audit = min(max(n_audit, 1 if rest.size else 0), rest.size)
    audit = np.sort(rng.choice(rest, size=n_audit, replace=False)) if n_audit else np.zeros(0, int)

    if progress:
        progress(f"predicted {active.size} modes; flagged {int(flagged.sum())}, audit", 0,
                 int(n_audit))
    rates = np.zeros((nT, nmodes))
    rates[:, active] = np.exp(mu)
    pred_audit = np.exp(mu[:, audit])

    deadline = None if max_exact_seconds is None else time.perf_counter() + max_exact_seconds
    t_audit = t_flag = 0.0
    done_a = np.ones(0, bool)
    if audit.size:
        ra, t_audit, done_a = exact_chunked(ctx, T, scalebroad, active[audit], precision, chunk,
                                            progress, "audit", ckpt, deadline)
        rates[:, active[audit]] = np.where(done_a[None, :], ra, rates[:, active[audit]])
    else:
        ra = np.zeros((nT, 0))
    fl = np.flatnonzero(flagged)
    done_f = np.ones(0, bool)
    if fl.size:
        rf, t_flag, done_f = exact_chunked(ctx, T, scalebroad, active[fl], precision, chunk,
                                           progress, "flagged", ckpt, deadline)
        rates[:, active[fl]] = np.where(done_f[None, :], rf, rates[:, active[fl]])
    rep["complete"] = bool(done_a.all() and done_f.all())
    rep["exact_done"] = {"audit": int(done_a.sum()), "flagged": int(done_f.sum())}

    # audit statistics: relative error of the predictions that were kept for every other mode
    if audit.size and done_a.any():
        ra_d, pa_d = ra[:, done_a], pred_audit[:, done_a]
        good = ra_d > 0
        rel = np.abs(pa_d[good] - ra_d[good]) / ra_d[good]
        z = np.abs(mu[:, audit][:, done_a][good] - np.log(ra_d[good])) / sig[:, audit][:, done_a][good]
        nzero = int((~good).sum())
        rep["audit_rel_err"] = {
            "median": float(np.median(rel)), "p90": float(np.quantile(rel, 0.9)),
            "p99": float(np.quantile(rel, 0.99)), "max": float(rel.max()),
            "mean": float(rel.mean()),
            "frac_within_10pct": float(np.sum(rel <= 0.1) / (rel.size + nzero)),
            "frac_within_2sigma": float(np.mean(z <= 2.0)), "n": int(rel.size)}
        rep["audit_zero_rate"] = nzero
    per_target = t_audit / max(int(done_a.sum()), 1)
    t_total = t_feat + t_pred + t_audit + t_flag
    rep.update({
        "flagged": int(fl.size), "flagged_frac": float(fl.size / max(active.size, 1)),
        "out_of_range": int(np.any(oor, axis=0).sum()), "audit": int(audit.size),
        "fallback_frac": float((fl.size + audit.size) / max(active.size, 1)),
        "seconds": {"features_and_3ph": t_feat, "inference": t_pred, "inference_device_ms": ms_net,
                    "audit_exact": t_audit, "flagged_exact": t_flag, "total": t_total},
        "exact_seconds_per_mode": per_target,
        "exact_all_modes_seconds_estimate": per_target * active.size,
        "speedup_vs_exact_estimate": (per_target * active.size / t_total) if t_total > 0 else None,
    })
    rep["audit_modes"] = active[audit].tolist()
    rep["flagged_modes"] = active[fl].tolist()
    return rates, rep
