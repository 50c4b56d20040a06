"""Write the oracle's expected values for the parity tests at the benchmarked sizes.

Calls only the FP64 CPU oracle (`oracle/`) on the seeded synthetic workloads (`synth/`);
nothing here touches the HIP library.  Each record stores a fingerprint of the inputs it was
computed from (SHA-256 of the grid, masses, lattice, modes and quartet list), so a test can
tell whether the workload it regenerates is bit-identical to the one the values belong to.

    python tests/golden/make_oracle_values.py [--threads N] [--only NAME]

Cases (every rate at every temperature, kept counts per channel):
  medium-8x8x8    the 8x8x8 second-shell workload (T = 300, 1000 K, scalebroad 1): complete
                  rates of 4 modes, the lowest-frequency non-Gamma acoustic mode among them
  large-16x16x16  the 16x16x16 workload (T = 300 K): counts of 8 modes at scalebroad 1, the
                  recombination and splitting rates of 3 of them at scalebroad 1, and the
                  complete rate of the one with the fewest kept processes at scalebroad 0.1
  cubic-10x10x10, wurtzite-8x8x6, layered-6x6x6
                  the three instances of the batched workload (T = 300, 700 K): counts of 8
                  modes and the complete rate of the one with the fewest kept processes
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from synth import configs  # noqa: E402

OUT = os.path.join(HERE, "oracle_values.json")


def fingerprint(inst) -> str:
    h = hashlib.sha256()
    for a in (np.asarray(inst.grid, dtype=np.int64), np.asarray(inst.cr.mass, dtype=np.float64),
              np.asarray(inst.cr.A, dtype=np.float64), np.asarray(inst.omega, dtype=np.float64),
              np.asarray(inst.vel, dtype=np.float64), np.asarray(inst.evec, dtype=np.complex128),
              np.asarray(inst.fc4.atoms, dtype=np.int32), np.asarray(inst.fc4.cells, dtype=np.int32),
              np.asarray(inst.fc4.phi, dtype=np.float64)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


INSTANCES = {
    "medium-8x8x8": synth.medium,
    "large-16x16x16": synth.large,
    "cubic-10x10x10": configs.cubic10,
    "wurtzite-8x8x6": configs.wurtzite,
    "layered-6x6x6": configs.layered,
}


def sample_modes(inst, k, seed):
    """k distinct active modes drawn with a seeded generator (Gamma acoustic modes excluded)."""
    om = np.asarray(inst.omega).reshape(-1)
    act = np.nonzero(om > 0)[0]
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(act, k, replace=False)).astype(np.int32)


def _run(m, inst, T, sb, mask, targets, want_rates, threads):
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    t0 = time.time()
    r, rch, c = oracle.rates4(m, T, sb, mask, dq, targets, want_rates=want_rates, nthreads=threads)
    print(f"  sb {sb} mask {mask} targets {list(map(int, targets))} rates={want_rates}: "
          f"{time.time() - t0:.1f} s", flush=True)
    rec = {"T": list(map(float, T)), "scalebroad": sb, "mask": mask,
           "targets": [int(x) for x in targets], "counts": c.tolist()}
    if want_rates:
        rec["rates"] = r.tolist()
        rec["rates_by_channel"] = rch.tolist()
    return rec


def make(name, threads):
    inst = INSTANCES[name]()
    m = oracle.Model.from_instance(inst)
    T = list(inst.T)
    out = {"fingerprint": fingerprint(inst), "cases": {}}
    print(name, flush=True)
    if name == "medium-8x8x8":
        om = np.asarray(inst.omega).reshape(-1)
        act = np.nonzero(om > 0)[0]
        low = int(act[np.argmin(om[act])])
        tg = np.unique(np.concatenate([[low], sample_modes(inst, 3, 1002)])).astype(np.int32)
        out["lowest_mode"] = low
        out["cases"]["full"] = _run(m, inst, T, 1.0, 7, tg, True, threads)
    elif name == "large-16x16x16":
        tg = sample_modes(inst, 8, 1003)
        cnt = _run(m, inst, T, 1.0, 7, tg, False, threads)
        out["cases"]["counts"] = cnt
        out["cases"]["pp_mm"] = _run(m, inst, T, 1.0, 5, tg[:3], True, threads)
        c01 = _run(m, inst, T, 0.1, 7, tg, False, threads)
        out["cases"]["counts_sb01"] = c01
        tot = np.asarray(c01["counts"]).sum(axis=1)
        one = tg[np.argmin(np.where(tot > 0, tot, np.iinfo(np.int64).max))]
        out["cases"]["full_sb01"] = _run(m, inst, T, 0.1, 7, np.array([one], np.int32), True, threads)
    else:
        seed = {"cubic-10x10x10": 1041, "wurtzite-8x8x6": 1042, "layered-6x6x6": 1043}[name]
        tg = sample_modes(inst, 8, seed)
        cnt = _run(m, inst, T, 1.0, 7, tg, False, threads)
        out["cases"]["counts"] = cnt
        tot = np.asarray(cnt["counts"]).sum(axis=1)
        one = tg[np.argmin(np.where(tot > 0, tot, np.iinfo(np.int64).max))]
        out["cases"]["full"] = _run(m, inst, T, 1.0, 7, np.array([one], np.int32), True, threads)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    names = [args.only] if args.only else list(INSTANCES)
    for name in names:
        data[name] = make(name, args.threads)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
