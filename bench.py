"""Benchmark of the four-phonon RTA rate kernel on one MI355X.

One step = the whole rate computation (occupations, per-target precontraction, fused
enumeration / window prefilter / contraction / accumulation kernel, ordered reduction) for
every mode of the 8x8x8 diamond-structure workload (3072 modes, second-shell FC4 with 1522
quartets, T = 300 and 1000 K, scalebroad 1, all three channels), inputs resident in HBM.

Prints one JSON line.  `value` is kept four-phonon processes per second.

``--surrogate`` runs the learned-surrogate workload instead: exact rates on sampled modes of
12x12x12 grids of 8 seeded force-constant draws (T from 100 to 1200 K) train the network;
inference covers every mode of a held-out 20x20x20 grid (48 000 modes) with exact fallback
on flagged modes and a 2% audit.  Its JSON line reports the audit's relative error, the
fallback rate and the speedup over the plain FP64 kernel.

``--batched`` runs the uneven-instance workload: a 2-atom cubic 10x10x10 grid, a 4-atom
wurtzite-like 8x8x6 grid and a 4-atom layered 6x6x6 grid at T = 300, 700 K in one
persistent graph-captured launch with the FP32 contraction and autotuned work shapes (q'
chunk, queue and list segments), timed against separate calls, with every rate compared to
the FP64 path.

``--batched-small`` runs 28 small instances (24 diamond-structure cells on 2x2x2 .. 4x4x4
grids and 4 three-atom cells) in one graph replay against one synchronous call each.

``--umklapp`` splits the 8x8x8 rates into normal and Umklapp processes (two class-restricted
calls beside the unrestricted one) and reports kernel times, counts and the Umklapp share.

``--wedge`` computes the 8x8x8 rates on the irreducible grid points under the diamond
structure's 48 point-group operations and compares them with the full grid.

``--phase-space`` computes the phase spaces P4 and WP4 (no force constants) of the 8x8x8
workload and times them against the rates.

``--large`` runs the 16x16x16 workload (24 576 modes) on a random subset of 512 target modes
in FP64 and with the FP32 contraction, and in FP64 at scalebroad 0.1.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6e12      # MI355X FP64 vector FLOP/s
PEAK_FP32_VALU = 157.3e12

# Counter readings of one FP64 k_rates launch on this workload, from the rocprofv3 summary
# named in "source" (FETCH_SIZE and WRITE_SIZE scaled by their readings for a plain kernel
# that reads and writes 256 MiB; SQ_INSTS_VALU, the FP64 FMA + MUL + ADD counters and
# SQ_INSTS_MFMA).  They are reported only while kernel_build_key() equals "build_key": the
# kernel sources without comments, the hipcc flags and the ROCm release they were taken
# with.  The chip issues at most one wave64 FP64 VALU instruction per CU per cycle: 256 CUs
# x 2.4 GHz.
COUNTERS_FP64 = {"build_key": "d8c1ba0d0838c13c", "source": "profiles/k_rates_diamond8x8x8_fp64.md",
                 "traffic_bytes": 889599669.0, "valu_insts": 373089497237.0,
                 "fp64_insts": 199695849085.0, "mfma_insts": 0.0}
VALU_ISSUE_PER_S = 256 * 2.4e9


def kernel_build_key():
    """sha256 (first 16 hex digits) of what the rate kernel's launches depend on: its sources
    and the host code that chooses their shapes (q' chunks, segments), with comments and
    blank lines removed (a comment edit does not invalidate the counter readings), the hipcc
    flags of the build, and the ROCm release."""
    import hashlib
    import re
    from paper_2104_04895_amd import build as hb
    h = hashlib.sha256()
    for f in ("fp4_kernels.hip", "fp4_device.h", "fp4_internal.h", "fp4_api.cpp"):
        with open(os.path.join(ROOT, "paper_2104_04895_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
        h.update("\n".join(ln for ln in lines if ln.strip()).encode())
    h.update(" ".join(hb.HIPCC_FLAGS).encode())
    try:
        with open("/opt/rocm/.info/version") as fh:
            h.update(fh.read().strip().encode())
    except OSError:
        h.update(b"unknown-rocm")
    return h.hexdigest()[:16]


def algorithmic_flops(stats, inst, n_pairs):
    """Algorithmic FLOPs of one main-kernel launch, the cheapest grouping of the arithmetic:
    W'' build 456 per combo per (lambda, lambda') pair, branch block 72 ng + 16 nb^3 per
    contracted block, Gamma 40 + 6 nT per kept process of ++ and --, and for +- per mirror
    pair 40 + 6 nT + 13 (the second member's dw and Gaussian), counting every +- process as a
    pair member, which slightly undercounts (the per-candidate window test is not
    credited)."""
    ng, nc, nb = inst["ng"], inst["nc"], inst["nb"]
    nT = inst["nT"]
    g = 40.0 + 6.0 * nT
    return (456.0 * nc * n_pairs
            + (72.0 * ng + 16.0 * nb ** 3) * stats["blocks"]
            + g * stats["processes_pp_mm"] + (g + 13.0) * 0.5 * stats["processes_pm"])


def groups_and_combos(fc4):
    g, c = set(), set()
    for n in range(fc4.n):
        i, j, k, l = (int(x) for x in fc4.atoms[n])
        Rj, Rk, Rl = (tuple(int(v) for v in fc4.cells[n, s]) for s in range(3))
        d = tuple(a - b for a, b in zip(Rk, Rl))
        a = tuple(x - y for x, y in zip(Rj, Rl))
        g.add((k, l, d))
        c.add((k, l, d, j, a))
    return len(g), len(c)


def surrogate_main(args):
    import synth
    from synth.fc3 import random_fc3
    import paper_2104_04895_amd as fp4
    from paper_2104_04895_amd import surrogate as S

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    tg = (args.train_grid,) * 3
    ig = (args.infer_grid,) * 3
    T_train = [100.0, 200.0, 400.0, 700.0, 1000.0, 1200.0]
    T_inf = [300.0, 700.0]

    def load(grid, seed):
        inst = synth.diamond_instance(grid, synth.configs.RC_SECOND, seed=seed)
        fc3 = random_fc3(inst.cr, synth.configs.RC_FIRST, np.random.default_rng(seed + 500))
        c = fp4.Context(0)
        c.load_instance(inst)        # dq = the library's default (|det B| / N)^(1/3)
        c.load_fc3(fc3.atoms, fc3.cells, fc3.phi)
        return inst, c

    ckpt = args.ckpt_dir
    model_prefix = os.path.join(ckpt, "surrogate") if ckpt else None
    if ckpt:
        os.makedirs(ckpt, exist_ok=True)
    if model_prefix and os.path.exists(model_prefix + ".npy") and os.path.exists(model_prefix + "_train.json"):
        # resumed pass: the trained network and its training record come from the checkpoint
        sur = S.Surrogate.load(model_prefix)
        with open(model_prefix + "_train.json") as f:
            training = json.load(f)
        log(f"loaded the trained surrogate from {model_prefix}")
    else:
        sur, training = None, None
    rng = np.random.default_rng(0)
    tr, ca = S.TrainSet(), S.TrainSet()
    t_train_exact = 0.0
    t0 = time.perf_counter()
    for d in range(args.draws if sur is None else 0):
        inst, c = load(tg, 1000 + d)
        modes = rng.permutation(inst.nmodes)
        n_tr = int(args.sample_frac * inst.nmodes)
        n_ca = max(8, n_tr // 5)
        if args.calib_draw and d == args.draws - 1:
            # the last draw is held out whole: it only calibrates sigma (draw-level calibration)
            X2, y2, te2 = S.collect(c, inst.omega, T_train, 1.0, modes[:n_tr])
            ca.add(X2, y2)
            te = 0.0
        else:
            X, y, te = S.collect(c, inst.omega, T_train, 1.0, modes[:n_tr])
            tr.add(X, y)
            te2 = 0.0
            if not args.calib_draw:
                X2, y2, te2 = S.collect(c, inst.omega, T_train, 1.0, modes[n_tr:n_tr + n_ca])
                ca.add(X2, y2)
        t_train_exact += te + te2
        c.close()
        log(f"draw {d}: exact modes in {te + te2:.1f} s")
    if sur is None:
        sur = S.Surrogate(seed=1)
        X, y = tr.arrays()
        t1 = time.perf_counter()
        loss = sur.fit(X, y, epochs=args.epochs, batch=256, lr=1e-3)
        t_fit = time.perf_counter() - t1
        kappa = sur.calibrate(*ca.arrays())
        log(f"trained on {len(y)} rows in {t_fit:.1f} s, loss {loss[0]:.3f} -> {loss[-1]:.3f}, "
            f"kappa {kappa:.2f}")
        training = {"rows": int(len(y)), "exact_seconds": t_train_exact, "fit_seconds": t_fit,
                    "loss_first": float(loss[0]), "loss_last": float(loss[-1]), "kappa": kappa,
                    "wall_seconds": time.perf_counter() - t0}
        if model_prefix:
            sur.save(model_prefix)
            with open(model_prefix + "_train.json", "w") as f:
                json.dump(training, f)
    seed = 1000 if not args.unseen_draw else 2000
    inst, c = load(ig, seed)
    log(f"inference grid {ig} ({inst.nmodes} modes) loaded; the exact fallback and audit follow")
    rates, rep = S.infer(sur, c, inst.omega, T_inf, flag_sigma=args.flag_sigma,
                         audit_frac=0.02, audit_seed=7, chunk=64,
                         progress=lambda what, done, tot: log(f"{what} exact {done}/{tot}"),
                         ckpt=ckpt, max_exact_seconds=args.max_exact_seconds)
    c.close()
    rep.pop("audit_modes")
    rep.pop("flagged_modes")
    out = {
        "metric": "surrogate 4ph rates: audit rel. err vs exact, fallback rate, speedup over the plain FP64 kernel",
        "value": rep["speedup_vs_exact_estimate"],
        "unit": "x (time of the exact FP64 kernel on all modes, estimated from the audit's "
                "per-mode time, over the whole surrogate pass)",
        "n_gpus": 1, "higher_is_better": True, "dtype": "bf16-inference/f64-exact",
        "data": "synthetic",
        "config": {"workload": f"diamond-structure 2-atom cell, second-shell FC4, first-shell FC3; "
                               f"train {args.draws} draws x {tg[0]}^3 grid ({args.sample_frac:.0%} of modes, "
                               f"T=100..1200 K); infer {ig[0]}^3 grid of "
                               + ("an unseen draw" if args.unseen_draw else "training draw 0")
                               + ", T=300,700 K",
                   "flag_sigma": args.flag_sigma, "audit_frac": 0.02, "epochs": args.epochs,
                   "sigma_calibration": "held-out draw" if args.calib_draw else "held-out modes"},
        "training": training,
        "report": rep,
    }
    print(json.dumps(out))
    sur.close()


def batched_main(args):
    """Uneven instances in one persistent graph-captured launch (FP32 contraction), against
    the same instances one call at a time, with every rate compared to the FP64 path."""
    from synth import configs
    import paper_2104_04895_amd as fp4

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    T = [300.0, 700.0]
    insts = [configs.cubic10(), configs.wurtzite(), configs.layered()]
    ctxs, tuned = [], []
    for inst in insts:
        c = fp4.Context(0)
        c.load_instance(inst)
        c.set_param(fp4.FP4_PARAM_PROFILE, 1)
        best, table = fp4.autotune_shapes(c, T, 1.0, 7, fp4.FP4_FP32, nsample=32)
        tuned.append({"instance": inst.name, "qchunk_qseg_lseg": list(best),
                      "ms_by_config": [[list(cfg), ms] for cfg, ms in table]})
        ctxs.append(c)
        log(f"{inst.name}: {inst.nmodes} modes, autotuned (q' chunk, queue, list) {best}")
    ref, t64, t32, procs = [], [], [], []
    for inst, c in zip(insts, ctxs):
        t0 = time.perf_counter()
        r, _, cnt = c.compute_rates4(T, 1.0, 7, fp4.FP4_FP64)
        t64.append(time.perf_counter() - t0)
        ref.append(r)
        procs.append(int(cnt.sum()))
        t0 = time.perf_counter()
        c.compute_rates4(T, 1.0, 7, fp4.FP4_FP32)
        t32.append(time.perf_counter() - t0)
        log(f"{inst.name}: FP64 {t64[-1]:.2f} s, FP32 {t32[-1]:.2f} s one call each")
    b = fp4.Batch(0)
    for c in ctxs:
        b.add(c)
    b.compute(T, 1.0, 7, fp4.FP4_FP32)            # builds and launches the graph once
    log("graph built; timing replays")
    times = []
    for k in range(args.steps):
        t0 = time.perf_counter()
        rb, cb = b.compute(T, 1.0, 7, fp4.FP4_FP32)
        times.append(time.perf_counter() - t0)
        log(f"replay {k}: {times[-1]:.2f} s (graph {b.last_timing()['ms_graph']:.1f} ms)")
    tm = b.last_timing()
    per = []
    for inst, r64, r32, cnt in zip(insts, ref, rb, cb):
        rel = np.abs(r32 - r64) / np.maximum(np.abs(r64), 1e-300)
        rel[r64 == 0] = 0.0
        per.append({"instance": inst.name, "modes": inst.nmodes, "nb": inst.nb,
                    "grid": list(inst.grid), "processes": int(cnt.sum()),
                    "max_rel_err_vs_fp64": float(rel.max()),
                    "median_rel_err_vs_fp64": float(np.median(rel[r64 > 0]))})
    total = sum(procs)
    t_batch = float(np.mean(times))
    out = {
        "metric": "batched uneven instances: 4ph processes/s in one persistent graph-captured launch (FP32 contraction)",
        "value": total / t_batch, "unit": "processes/s", "n_gpus": 1, "steps": args.steps,
        "higher_is_better": True, "dtype": "f32-contraction/f64", "data": "synthetic",
        "config": {"workload": "2-atom cubic 10x10x10 (6 branches), 4-atom wurtzite-like 8x8x6 "
                               "(12), 4-atom layered rhombohedral 6x6x6 (12); T=300,700 K",
                   "instances": per, "autotune": tuned},
        "seconds": {"batch_graph_mean": t_batch, "batch_graph_device_ms": tm["ms_graph"],
                    "separate_fp32_calls_total": float(sum(t32)),
                    "separate_fp64_calls_total": float(sum(t64))},
        "speedup_batch_vs_separate_fp32": float(sum(t32)) / t_batch,
        "speedup_batch_fp32_vs_separate_fp64": float(sum(t64)) / t_batch,
    }
    print(json.dumps(out))
    b.close()
    for c in ctxs:
        c.close()


def batched_small_main(args):
    """Many small uneven instances (the regime a single persistent launch is for): 24 diamond
    cells on 2x2x2 .. 4x4x4 grids plus 4 three-atom cells, FP32 contraction, T = 300/700 K;
    one graph replay against one synchronous call per instance (both return host rates)."""
    from synth import configs
    import paper_2104_04895_amd as fp4

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    T = [300.0, 700.0]
    grids = [(2, 2, 2), (3, 3, 3), (2, 3, 4), (4, 4, 3), (4, 4, 4), (3, 2, 2)]
    insts = [configs.diamond_instance(grids[i % len(grids)], configs.RC_SECOND, 100 + i,
                                      tuple(T), fc4_seed=7, name=f"diamond-{i}")
             for i in range(24)]
    insts += [configs.three_atom(seed=44, grid=g) for g in [(2, 2, 2), (2, 2, 3), (3, 2, 2), (2, 3, 2)]]
    ctxs = []
    for inst in insts:
        c = fp4.Context(0)
        c.load_instance(inst)
        ctxs.append(c)
    ref, procs = [], []
    for c in ctxs:                                    # FP64 reference, and warm every path
        r, _, cnt = c.compute_rates4(T, 1.0, 7, fp4.FP4_FP64)
        ref.append(r)
        procs.append(int(cnt.sum()))
        c.compute_rates4(T, 1.0, 7, fp4.FP4_FP32)
    sep = []
    for k in range(args.steps):
        t0 = time.perf_counter()
        for c in ctxs:
            c.compute_rates4(T, 1.0, 7, fp4.FP4_FP32)
        sep.append(time.perf_counter() - t0)
    log(f"{len(ctxs)} instances, separate calls: {np.mean(sep) * 1e3:.1f} ms per pass")
    b = fp4.Batch(0)
    for c in ctxs:
        b.add(c)
    b.compute(T, 1.0, 7, fp4.FP4_FP32)                # builds the graph
    times = []
    for k in range(args.steps):
        t0 = time.perf_counter()
        rb, cb = b.compute(T, 1.0, 7, fp4.FP4_FP32)
        times.append(time.perf_counter() - t0)
    log(f"graph replay: {np.mean(times) * 1e3:.1f} ms per pass")
    err = 0.0
    for r64, r32 in zip(ref, rb):
        rel = np.abs(r32 - r64) / np.maximum(np.abs(r64), 1e-300)
        rel[r64 == 0] = 0.0
        err = max(err, float(rel.max()))
    t_b, t_s = float(np.mean(times)), float(np.mean(sep))
    out = {
        "metric": "batched small instances: 4ph processes/s in one persistent graph-captured launch (FP32 contraction)",
        "value": sum(procs) / t_b, "unit": "processes/s", "n_gpus": 1, "steps": args.steps,
        "higher_is_better": True, "dtype": "f32-contraction/f64", "data": "synthetic",
        "config": {"workload": "24 diamond-structure cells (second-shell FC4) on 2x2x2..4x4x4 "
                               "grids and 4 three-atom cells on 12-point grids; T=300,700 K",
                   "instances": len(insts), "modes": int(sum(i.nmodes for i in insts)),
                   "processes": int(sum(procs))},
        "seconds": {"graph_replay_mean": t_b, "graph_device_ms": b.last_timing()["ms_graph"],
                    "separate_calls_mean": t_s},
        "speedup_batch_vs_separate": t_s / t_b,
        "max_rel_err_vs_fp64": err,
    }
    print(json.dumps(out))
    b.close()
    for c in ctxs:
        c.close()


def umklapp_main(args):
    """Normal / Umklapp split of the 8x8x8 workload (FP64, T = 300, 1000 K): the
    unrestricted call and the two class-restricted calls (FP4_PARAM_QCLASS 1 and 2), their
    kernel times, process counts and Umklapp share, and the check that the classes add up."""
    import synth
    import paper_2104_04895_amd as fp4

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    inst = synth.medium()
    ctx = fp4.Context(0)
    ctx.load_instance(inst)
    ctx.set_param(fp4.FP4_PARAM_PROFILE, 1)
    res = {}
    for name, cls in (("all", 0), ("normal", 1), ("umklapp", 2)):
        ctx.set_param(fp4.FP4_PARAM_QCLASS, cls)
        r, rch, cnt = ctx.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64, by_channel=True)
        tm = ctx.last_timing()
        res[name] = (r, rch, cnt, tm["ms_main"], ctx.last_stats()["blocks"])
        log(f"{name}: kernel {tm['ms_main']:.0f} ms, {int(cnt.sum())} processes")
    r, rch, cnt, ms, blk = res["all"]
    rn, rchn, cntn, msn, blkn = res["normal"]
    ru, rchu, cntu, msu, blku = res["umklapp"]
    act = r > 0
    share = np.zeros_like(r)
    share[act] = ru[act] / r[act]
    out = {
        "metric": "normal/Umklapp split of the 4ph rates: kernel time per class and Umklapp share",
        "value": float(ms / 1e3), "unit": "s (unrestricted FP64 kernel)", "n_gpus": 1,
        "higher_is_better": False, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "diamond-structure 2-atom cell, 8x8x8 grid (3072 modes), "
                               "second-shell FC4, T=300,1000 K, scalebroad 1"},
        "kernel_ms": {"all": ms, "normal": msn, "umklapp": msu},
        "contracted_blocks": {"all": int(blk), "normal": int(blkn), "umklapp": int(blku)},
        "processes": {"all": int(cnt.sum()), "normal": int(cntn.sum()), "umklapp": int(cntu.sum())},
        "processes_by_channel": {"normal": [int(x) for x in cntn.sum(0)],
                                 "umklapp": [int(x) for x in cntu.sum(0)]},
        "umklapp_share_of_rate": {"median": float(np.median(share[act])),
                                  "min": float(share[act].min()), "max": float(share[act].max())},
        "classes_add_up": {"counts_exact": bool(np.array_equal(cntn + cntu, cnt)),
                           "max_rel_diff_rates": float(np.max(np.abs(rn + ru - r)[act] / r[act]))},
    }
    print(json.dumps(out))
    ctx.close()


def wedge_main(args):
    """The 8x8x8 workload (FP64) on the irreducible grid points under the 48 point-group
    operations of the diamond structure, against the full-grid call averaged over degenerate
    branches."""
    import synth
    import paper_2104_04895_amd as fp4

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    inst = synth.medium()
    A = np.asarray(inst.cr.A, dtype=np.float64)
    Ai = np.linalg.inv(A)
    rots = np.unique(np.array([np.rint(A @ np.asarray(T) @ Ai).astype(np.int32)
                               for T, _ in inst.cr.ops]).reshape(-1, 9), axis=0)
    ctx = fp4.Context(0)
    ctx.load_instance(inst)
    t0 = time.perf_counter()
    r_full, _, _ = ctx.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)
    t_full = time.perf_counter() - t0
    t0 = time.perf_counter()
    r_w, _, nirr = ctx.compute_rates4_wedge(inst.T, 1.0, 7, fp4.FP4_FP64, rots)
    t_w = time.perf_counter() - t0
    log(f"full grid {t_full:.2f} s, wedge ({nirr} of {inst.nq} points) {t_w:.2f} s")
    w = inst.omega.reshape(-1, inst.nb)
    ref = r_full.copy()
    for iq in range(w.shape[0]):
        j = 0
        while j < inst.nb:
            e = j + 1
            while e < inst.nb and abs(w[iq, e] - w[iq, j]) <= 1e-9 * max(abs(w[iq, j]), 1e-30):
                e += 1
            ref[:, iq * inst.nb + j:iq * inst.nb + e] = r_full[:, iq * inst.nb + j:iq * inst.nb + e].mean(1, keepdims=True)
            j = e
    act = ref > 0
    out = {
        "metric": "4ph rates on the irreducible wedge: time to solution against the full grid",
        "value": t_full / t_w, "unit": "x (full-grid wall time / wedge wall time)", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "diamond-structure 2-atom cell, 8x8x8 grid (3072 modes), "
                               "second-shell FC4, T=300,1000 K, scalebroad 1, 48 point-group operations"},
        "irreducible_points": int(nirr), "grid_points": int(inst.nq),
        "seconds": {"full_grid": t_full, "wedge": t_w},
        "max_rel_diff_vs_full_grid_degenerate_averaged": float(np.max(np.abs(r_w - ref)[act] / ref[act])),
    }
    print(json.dumps(out))
    ctx.close()


def phase_space_main(args):
    """Phase spaces of the 8x8x8 workload (no force constants used): P4 and WP4 with the
    kept-process counts, timed against the rate call (the quick estimate of the cost of the
    four-phonon sum the phase spaces serve for)."""
    import synth
    import paper_2104_04895_amd as fp4

    inst = synth.medium()
    ctx = fp4.Context(0)
    ctx.load_instance(inst)
    ctx.set_param(fp4.FP4_PARAM_PROFILE, 1)
    res = {}
    for name, kind in (("rates", 0), ("wp4", 1), ("p4", 2)):
        ctx.set_param(fp4.FP4_PARAM_PHASE_SPACE, kind)
        v, _, cnt = ctx.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)
        res[name] = (v, cnt, ctx.last_timing()["ms_main"])
        print(f"# {name}: kernel {res[name][2]:.0f} ms", file=sys.stderr, flush=True)
    act = res["p4"][0][0] > 0
    out = {
        "metric": "four-phonon phase spaces P4 / WP4 and kept-process counts: kernel time against the rates",
        "value": res["rates"][2] / res["p4"][2], "unit": "x (rate kernel ms / P4 kernel ms)",
        "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "diamond-structure 2-atom cell, 8x8x8 grid (3072 modes), "
                               "T=300,1000 K, scalebroad 1 (no force constants used)"},
        "kernel_ms": {k: res[k][2] for k in res},
        "counts_equal_to_rates_call": bool(np.array_equal(res["p4"][1], res["rates"][1])
                                          and np.array_equal(res["wp4"][1], res["rates"][1])),
        "p4_ps": {"median": float(np.median(res["p4"][0][0][act])), "max": float(res["p4"][0][0].max())},
        "wp4_300K_ps5": {"median": float(np.median(res["wp4"][0][0][act])),
                         "max": float(res["wp4"][0][0].max())},
    }
    print(json.dumps(out))
    ctx.close()


def large_leg(subset, with_sb01=True):
    """16x16x16 grid (24 576 modes), second-shell FC4, T = 300 K: a seeded random subset of
    `subset` target modes in FP64 and with the FP32 contraction, every rate of the FP32 path
    compared with the FP64 path, and (with_sb01) in FP64 at scalebroad 0.1; full-grid times
    are extrapolated from the subset."""
    import synth
    import paper_2104_04895_amd as fp4

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    inst = synth.large()
    ctx = fp4.Context(0)
    ctx.load_instance(inst)
    ctx.set_param(fp4.FP4_PARAM_PROFILE, 1)
    rng = np.random.default_rng(1003)
    act = np.flatnonzero(inst.omega.reshape(-1) > 0)
    targets = np.sort(rng.choice(act, size=subset, replace=False)).astype(np.int32)
    log(f"16^3 workload: {inst.nmodes} modes, {inst.fc4.n} quartets, subset {len(targets)}")
    out = {}
    r64 = None
    for name, prec in (("fp64", fp4.FP4_FP64), ("fp32", fp4.FP4_FP32)):
        t0 = time.perf_counter()
        r, _, cnt = ctx.compute_rates4(inst.T, 1.0, 7, prec, targets)
        wall = time.perf_counter() - t0
        tm = ctx.last_timing()
        out[name] = {"wall_s": wall, "kernel_ms": tm["ms_main"], "processes": int(cnt.sum()),
                     "processes_per_s": int(cnt.sum()) / (tm["ms_main"] / 1e3)}
        if r64 is None:
            r64 = r
        else:
            rel = np.abs(r - r64) / np.maximum(np.abs(r64), 1e-300)
            rel[r64 == 0] = 0.0
            out[name]["max_rel_err_vs_fp64_path"] = float(rel.max())
            out[name]["median_rel_err_vs_fp64_path"] = float(np.median(rel[r64 > 0]))
        log(f"{name}: {wall:.1f} s, kernel {tm['ms_main']:.0f} ms, {int(cnt.sum())} processes")
    if with_sb01:
        # the paper's cost figure is quoted for a 16x16x16 grid at scalebroad 0.1: same subset
        t0 = time.perf_counter()
        _, _, cnt01 = ctx.compute_rates4(inst.T, 0.1, 7, fp4.FP4_FP64, targets)
        tm = ctx.last_timing()
        out["fp64_sb0.1"] = {"wall_s": time.perf_counter() - t0, "kernel_ms": tm["ms_main"],
                             "processes": int(cnt01.sum()),
                             "full_grid_seconds_extrapolated": tm["ms_main"] / 1e3 * len(act) / len(targets)}
        log(f"fp64 sb 0.1: kernel {tm['ms_main']:.0f} ms, {int(cnt01.sum())} processes")
    full = out["fp64"]["kernel_ms"] / 1e3 * len(act) / len(targets)
    ctx.close()
    return {
        "metric": "4ph processes/sec and rates time-to-solution; FP64 vs mixed at stated rel. err",
        "value": out["fp64"]["processes_per_s"], "unit": "processes/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"diamond-structure 2-atom cell, 16x16x16 grid (24576 modes), "
                               f"second-shell FC4, T=300 K, sb 1, random subset of {len(targets)} "
                               f"target modes (seed 1003)"},
        "paths": out,
        "full_grid_fp64_seconds_extrapolated": full,
        "fp32_speedup": out["fp64"]["kernel_ms"] / out["fp32"]["kernel_ms"],
    }


def large_main(args):
    print(json.dumps(large_leg(args.subset)))


def large_full_main(args):
    """16x16x16 grid (24 576 modes), second-shell FC4, T = 300 K, scalebroad 1: every active
    mode, in FP64 and with the FP32 contraction, in calls of `chunk` target modes (each call
    logged, so a long run shows progress); the rates of the two paths are compared mode by
    mode.  Time = sum of the calls' main-kernel times (HIP events) and their wall time."""
    import synth
    import paper_2104_04895_amd as fp4

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    inst = synth.large()
    ctx = fp4.Context(0)
    ctx.load_instance(inst)
    ctx.set_param(fp4.FP4_PARAM_PROFILE, 1)
    act = np.flatnonzero(inst.omega.reshape(-1) > 0).astype(np.int32)
    chunk = args.full_chunk
    out, rates = {}, {}
    for name, prec in (("fp64", fp4.FP4_FP64), ("fp32", fp4.FP4_FP32)):
        ms, wall, procs = 0.0, 0.0, 0
        r_all = np.zeros((len(inst.T), act.size))
        for a in range(0, act.size, chunk):
            tg = act[a:a + chunk]
            t0 = time.perf_counter()
            r, _, cnt = ctx.compute_rates4(inst.T, 1.0, 7, prec, tg)
            wall += time.perf_counter() - t0
            ms += ctx.last_timing()["ms_main"]
            procs += int(cnt.sum())
            r_all[:, a:a + chunk] = r
            log(f"{name}: {min(a + chunk, act.size)}/{act.size} modes, kernel {ms / 1e3:.1f} s")
        rates[name] = r_all
        out[name] = {"kernel_s": ms / 1e3, "wall_s": wall, "processes": procs,
                     "processes_per_s": procs / (ms / 1e3)}
    r64, r32 = rates["fp64"], rates["fp32"]
    rel = np.abs(r32 - r64) / np.maximum(np.abs(r64), 1e-300)
    rel[r64 == 0] = 0.0
    out["fp32"]["max_rel_err_vs_fp64_path"] = float(rel.max())
    out["fp32"]["median_rel_err_vs_fp64_path"] = float(np.median(rel[r64 > 0]))
    ctx.close()
    print(json.dumps({
        "metric": "4ph processes/sec and rates time-to-solution; FP64 vs mixed at stated rel. err",
        "value": out["fp64"]["processes_per_s"], "unit": "processes/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"diamond-structure 2-atom cell, 16x16x16 grid (24576 modes), "
                               f"second-shell FC4, T=300 K, sb 1, every active mode "
                               f"({act.size}) in calls of {chunk}"},
        "paths": out, "fp32_speedup": out["fp64"]["kernel_s"] / out["fp32"]["kernel_s"]}))


def mfma_probe_main(args):
    """Matrix cores against vector units on this GPU (fp4_probe_matrix_rates), and what that
    means for the branch-block products of the rate kernel (H = E3 F, V = H E4^T, 6x6 complex
    per block for the 2-atom cell): packed two blocks per 16x16 tile (the only sharing the
    per-block operands allow), the complex products take 4 real products each, K = 6 padded to
    the instruction's K.  Useful flops per tile: 2 blocks x 432 complex MACs x 8."""
    import paper_2104_04895_amd as fp4
    r = fp4.probe_matrix_rates(0)
    useful = 2 * 432 * 8.0
    issued_fp64 = 2 * 4 * 2 * (2 * 16 * 16 * 4)        # H and V, 4 real products, 2 k-steps
    issued_bf16 = 2 * 4 * 3 * 1 * (2 * 16 * 16 * 32)   # H and V, 4 products, 3-product split
    util64, util16 = useful / issued_fp64, useful / issued_bf16
    out = {
        "metric": "matrix cores vs vector units: measured TFLOP/s and the branch-block product placement",
        "value": r["fp64_mfma_16x16x4"] / r["fp64_valu_fma"], "unit": "x (FP64 MFMA / FP64 VALU rate)",
        "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
        "measured_tflops": r,
        "overlap": {
            "fp64_mixed_over_mean_of_halves": r["fp64_half_mfma_half_valu"] / (0.5 * (r["fp64_mfma_16x16x4"] + r["fp64_valu_fma"])),
            "bf16_mixed_over_mean_of_halves": r["bf16_half_mfma_half_fp32_valu"] / (0.5 * (r["bf16_mfma_16x16x32"] + r["fp32_valu_fma"]))},
        "block_product": {
            "tile_utilisation_fp64_mfma": util64, "tile_utilisation_bf16x3_mfma": util16,
            "effective_tflops_fp64_mfma": r["fp64_mfma_16x16x4"] * util64,
            "effective_tflops_bf16x3_mfma": r["bf16_mfma_16x16x32"] * util16,
            "vector_fp64_tflops": r["fp64_valu_fma"], "vector_fp32_tflops": r["fp32_valu_fma"]},
    }
    print(json.dumps(out))


def cpu_baseline_leg(inst, dq, gpu_proc_per_s):
    """The oracle, as it stands, on the host cores: 8 target modes stratified by frequency
    (evenly spaced ranks among the active modes) x 32 evenly spaced partner points q' of the
    8x8x8 workload, both temperatures, all channels; scaled to processes/s."""
    import oracle
    m = oracle.Model.from_instance(inst)
    om = inst.omega.reshape(-1)
    act = np.flatnonzero(om > 0)
    order = act[np.argsort(om[act], kind="stable")]
    targets = order[np.linspace(0, len(order) - 1, 8).round().astype(int)].astype(np.int32)
    q1 = np.arange(0, inst.nq, inst.nq // 32)
    t1 = time.perf_counter()
    _, c_o = oracle.rates4_partners(m, inst.T, inst.scalebroad, inst.mask, dq, targets, q1)
    dt = time.perf_counter() - t1
    nproc = int(c_o.sum())
    return {"value": nproc / dt, "unit": "processes/s", "cores": oracle.max_threads(),
            "kind": "oracle", "host_cpus": os.cpu_count(),
            "sample": f"8 target modes stratified by frequency x {len(q1)} of {inst.nq} partner "
                      f"q' points of the 8x8x8 workload, both temperatures, all channels "
                      f"({nproc} processes, {dt:.1f} s)",
            "gpu_over_cpu": gpu_proc_per_s / (nproc / dt)}


def small_oracle_leg(fp4):
    """The small 3x3x3 workload (162 modes, first-shell FC4, 300 K): the complete oracle on 1
    thread and on all host threads against the library's synchronous call."""
    import oracle
    import synth
    inst = synth.small()
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    m = oracle.Model.from_instance(inst)
    nall = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.rates4(m, inst.T, 1.0, 7, dq, nthreads=nall)
    t_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    r1, _, c1 = oracle.rates4(m, inst.T, 1.0, 7, dq, nthreads=1)
    t_one = time.perf_counter() - t0
    oracle.rates4(m, inst.T, 1.0, 1, dq, targets=[3], want_rates=False, nthreads=nall)  # restores
    with fp4.Context(0) as c:
        c.load_instance(inst, dq=dq)
        c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)       # warm
        t0 = time.perf_counter()
        r, _, cnt = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)
        t_gpu = time.perf_counter() - t0
    rel = np.abs(r - r1) / np.maximum(np.abs(r1), 1e-300)
    return {"workload": "diamond-structure 3x3x3 (162 modes), first-shell FC4 (58 quartets), 300 K",
            "processes": int(c1.sum()), "oracle_s_1_thread": t_one, "oracle_s_all_threads": t_all,
            "oracle_threads": nall, "gpu_sync_call_s": t_gpu,
            "counts_equal": bool(np.array_equal(cnt, c1)), "max_rel_err_fp64": float(rel.max())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 side measurement")
    ap.add_argument("--no-large", action="store_true", help="skip the 16x16x16 subset leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="before the steps, run one elementwise pass that reads and writes "
                         "256 MiB (calibrates hardware traffic counters)")
    ap.add_argument("--surrogate", action="store_true", help="run the learned-surrogate workload")
    ap.add_argument("--large", action="store_true",
                    help="16x16x16 workload on a random subset of target modes, FP64 and FP32")
    ap.add_argument("--subset", type=int, default=512)
    ap.add_argument("--large-full", action="store_true",
                    help="every mode of the 16x16x16 grid, FP64 and FP32 (about 11 minutes)")
    ap.add_argument("--full-chunk", type=int, default=2048)
    ap.add_argument("--batched", action="store_true",
                    help="run the batched uneven-instance workload (one graph-captured launch)")
    ap.add_argument("--batched-small", action="store_true",
                    help="run the many-small-instances batched workload")
    ap.add_argument("--umklapp", action="store_true",
                    help="normal / Umklapp split of the 8x8x8 workload")
    ap.add_argument("--phase-space", action="store_true",
                    help="phase spaces P4 / WP4 of the 8x8x8 workload against the rates")
    ap.add_argument("--wedge", action="store_true",
                    help="8x8x8 workload on the irreducible grid points against the full grid")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="measure matrix-core against vector-unit rates (branch-block placement)")
    ap.add_argument("--train-grid", type=int, default=12)
    ap.add_argument("--infer-grid", type=int, default=20)
    ap.add_argument("--draws", type=int, default=8)
    ap.add_argument("--sample-frac", type=float, default=0.1)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--flag-sigma", type=float, default=0.15)
    ap.add_argument("--unseen-draw", action="store_true")
    ap.add_argument("--calib-draw", action="store_true",
                    help="calibrate sigma on a whole held-out draw instead of held-out modes")
    ap.add_argument("--ckpt-dir", default=None,
                    help="surrogate: keep the trained network and every finished exact chunk "
                         "here, and resume from what is there")
    ap.add_argument("--max-exact-seconds", type=float, default=None,
                    help="surrogate: start no new exact chunk after this many seconds of the "
                         "inference pass (resume later with the same --ckpt-dir)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the rate kernel runs on a single MI355X and "
              f"--gpus {args.gpus} is not supported (multi-GPU sharding is a design note).",
              file=sys.stderr)
        sys.exit(2)
    if args.mfma_probe:
        mfma_probe_main(args)
        return
    if args.surrogate:
        surrogate_main(args)
        return
    if args.batched:
        batched_main(args)
        return
    if args.batched_small:
        batched_small_main(args)
        return
    if args.umklapp:
        umklapp_main(args)
        return
    if args.wedge:
        wedge_main(args)
        return
    if args.phase_space:
        phase_space_main(args)
        return
    if args.large_full:
        large_full_main(args)
        return
    if args.large:
        large_main(args)
        return

    import torch
    import synth
    import paper_2104_04895_amd as fp4

    t_setup = time.time()
    inst = synth.medium()
    dq = (abs(np.linalg.det(inst.cr.B)) / inst.nq) ** (1.0 / 3.0)
    ng, nc = groups_and_combos(inst.fc4)
    nmodes = inst.nmodes
    nT = len(inst.T)
    dev = torch.device("cuda:0")
    ctx = fp4.Context(0)
    ctx.load_instance(inst, dq=dq)
    ctx.set_param(fp4.FP4_PARAM_PROFILE, 1)
    prec = fp4.FP4_FP64 if args.precision == "fp64" else fp4.FP4_FP32
    d_rates = torch.empty((nT, nmodes), dtype=torch.float64, device=dev)
    d_counts = torch.empty((nmodes, 3), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(precision):
        ctx.compute_rates4_async(inst.T, inst.scalebroad, inst.mask, precision,
                                 stream.cuda_stream, d_rates.data_ptr(), 0, d_counts.data_ptr())

    if args.copy_probe:
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step(prec)
    torch.cuda.synchronize()
    print(f"# setup {time.time() - t_setup:.1f}s; timing {args.steps} steps", file=sys.stderr, flush=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    main_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        step(prec)
        main_ms.append(ctx.last_timing()["ms_main"])
        print(f"# step {k} main kernel {main_ms[-1]:.1f} ms", file=sys.stderr, flush=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_events = ev0.elapsed_time(ev1)
    ms_per_step = ms_events / args.steps
    counts = d_counts.cpu().numpy()
    processes = int(counts.sum())
    rates64 = d_rates.cpu().numpy().copy()

    # candidates: active targets x active partner modes^2 x nb x enabled channels
    act = int((inst.omega.reshape(-1) > 0).sum())
    nch = bin(inst.mask).count("1")
    # per active target: active lambda' x (N q'' x nb j'') x nb j''' per channel
    candidates = act * act * inst.nq * inst.nb * inst.nb * nch
    stats = {"processes": processes, "candidates": candidates,
             "processes_pp_mm": int(counts[:, 0].sum() + counts[:, 2].sum()),
             "processes_pm": int(counts[:, 1].sum())}
    lib_stats = ctx.last_stats()
    stats["blocks"] = lib_stats["blocks"]
    n_pairs = act * act
    flops = algorithmic_flops(stats, {"ng": ng, "nc": nc, "nb": inst.nb, "nT": nT}, n_pairs)
    t_main = float(np.mean(main_ms)) / 1e3
    peak = PEAK_FP64_VALU if prec == fp4.FP4_FP64 else PEAK_FP32_VALU
    achieved = flops / t_main
    counters = (prec == fp4.FP4_FP64 and COUNTERS_FP64["build_key"] is not None
                and kernel_build_key() == COUNTERS_FP64["build_key"])
    traffic = COUNTERS_FP64["traffic_bytes"] if counters else None

    extras = {
        "candidates_per_s": candidates / (ms_per_step / 1e3),
        "candidates_per_step": candidates,
        "contracted_blocks_per_step": stats["blocks"],
        "hbm_gb_per_s": (traffic / t_main / 1e9) if traffic else None,
        "counters_source": COUNTERS_FP64["source"] if counters else None,
        "kernel_build_key": kernel_build_key(),
    }
    if counters:
        extras["valu"] = {"insts_per_launch": COUNTERS_FP64["valu_insts"],
                          "issue_frac": COUNTERS_FP64["valu_insts"] / (t_main * VALU_ISSUE_PER_S),
                          "fp64_fma_mul_add_share": COUNTERS_FP64["fp64_insts"] / COUNTERS_FP64["valu_insts"]}
        # matrix-core instructions issued by the rate kernel (SQ_INSTS_VALU_MFMA_* counters)
        extras["mfma_insts_per_launch"] = COUNTERS_FP64["mfma_insts"]
    # time to solution: the synchronous call, rates and counts copied back to the host
    t0 = time.perf_counter()
    ctx.compute_rates4(inst.T, inst.scalebroad, inst.mask, prec)
    extras["time_to_solution_s"] = time.perf_counter() - t0
    if not args.no_fp32 and prec == fp4.FP4_FP64:
        step(fp4.FP4_FP32)
        torch.cuda.synchronize()
        ms32 = ctx.last_timing()["ms_main"]
        r32 = d_rates.cpu().numpy()
        rel = np.abs(r32 - rates64) / np.maximum(np.abs(rates64), 1e-300)
        rel[rates64 == 0] = 0.0
        extras["fp32_contraction"] = {"ms_main_kernel": ms32, "speedup_vs_fp64_main": t_main * 1e3 / ms32,
                                      "max_rel_err_vs_fp64_path": float(rel.max()),
                                      "median_rel_err_vs_fp64_path": float(np.median(rel[rates64 > 0]))}

    if not args.no_large:
        # the 16x16x16 workload (the paper's BAs grid) on a 512-mode subset, FP64 and FP32
        print("# 16x16x16 subset leg", file=sys.stderr, flush=True)
        extras["large_16cubed_subset"] = large_leg(512, with_sb01=False)

    cpu = None
    if not args.no_cpu_baseline:
        print("# CPU baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline_leg(inst, dq, processes / (ms_per_step / 1e3))
        extras["small_3cubed_oracle"] = small_oracle_leg(fp4)

    out = {
        "metric": "4ph processes/sec and rates time-to-solution; FP64 vs mixed at stated rel. err",
        "value": processes / (ms_per_step / 1e3),
        "unit": "processes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == fp4.FP4_FP64 else "f32-contraction/f64",
        "data": "synthetic",
        "config": {"workload": "diamond-structure 2-atom cell, 8x8x8 Gamma grid (3072 modes), "
                               "second-shell FC4 (1522 quartets), T=300,1000 K, scalebroad 1, "
                               "channels ++,+-,--",
                   "modes": nmodes, "temperatures": list(inst.T), "processes_per_step": processes,
                   "wall_s_timed": wall},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "kernel": "k_rates", "kernel_ms": t_main * 1e3,
                     "algorithmic_flops": flops},
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
