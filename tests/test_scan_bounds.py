"""The frequency bounds the rate kernel uses to skip work never drop a kept process.

The kernel scans q'' of the ++ and -- channels in ascending order of the lowest active
frequency at q'' and stops at a threshold, culls a block (q'', q''') from the frequency
ranges and largest speeds at both points, and a row (q'', j'') from the frequency range and
largest speed at q'''.  Both rest on the same inequality: a kept process has
|dw| <= sqrt(c_win) |v'' - v'''| (the window of the adaptive Gaussian, Sec. 2.4 / App. B),
hence |dw| <= sqrt(c_win) (|v''| + v_max(q''')) <= 2 sqrt(c_win) v_max.  Here every candidate
process of the 3x3x3 workload is tested with the exact FP64 predicate (same operation order
as the stand-alone process test), and every kept one is checked against the bounds, with a
relative slack of 1e-12 only (the kernel applies them with 1e-6).
"""
import numpy as np
import pytest

import oracle
import synth


def _grid_fold(grid):
    g = np.array(grid)
    n = np.stack(np.meshgrid(*[np.arange(x) for x in grid], indexing="ij"), -1)
    n = n.transpose(2, 1, 0, 3).reshape(-1, 3)          # iq = n1 + g0 (n2 + g1 n3)
    def fold(m):
        m = np.mod(m, g)
        return m[..., 0] + g[0] * (m[..., 1] + g[1] * m[..., 2])
    return n, fold


@pytest.mark.parametrize("sb", [1.0, 2.0])
def test_kept_processes_respect_the_scan_and_cull_bounds(sb):
    inst = synth.small()
    grid = inst.grid
    w = np.asarray(inst.omega, dtype=np.float64).reshape(-1, inst.nb)
    v = np.asarray(inst.vel, dtype=np.float64).reshape(-1, inst.nb, 3)
    N, nb = w.shape
    act = w > 0
    dq = oracle.default_dq(inst.cr.A, grid)
    c_win = (2.0 * sb * dq) ** 2
    sq = np.sqrt(c_win)
    speed = np.sqrt((v ** 2).sum(-1))
    w_lo, w_hi, v_hi = w[act].min(), w[act].max(), speed[act].max()
    wmin_q = np.where(act, w, np.inf).min(1)
    wmax_q = np.where(act, w, -np.inf).max(1)
    vmax_q = np.where(act, speed, 0.0).max(1)
    n, fold = _grid_fold(grid)
    kept_total = {0: 0, 2: 0}
    for ch, (s1, s2) in {0: (1, 1), 2: (-1, -1)}.items():
        for iq in range(N):
            for iq1 in range(N):
                iq2 = np.arange(N)
                iq3 = fold(n[iq] + s1 * n[iq1] + s2 * n[iq2])
                # [j, j1, q'', j2, j3]
                W0 = w[iq][:, None, None, None, None]
                W1 = w[iq1][None, :, None, None, None]
                W2 = w[iq2][None, None, :, :, None]
                W3 = w[iq3][None, None, :, None, :]
                aw = W0 + W1 if s1 > 0 else W0 - W1
                bw = aw + W2 if s2 > 0 else aw - W2
                dw = bw - W3
                d = v[iq2][:, :, None, :] - v[iq3][:, None, :, :]
                s2v = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
                live = (act[iq][:, None, None, None, None] & act[iq1][None, :, None, None, None]
                        & act[iq2][None, None, :, :, None] & act[iq3][None, None, :, None, :])
                keep = live & (dw * dw <= c_win * s2v[None, None])
                if not keep.any():
                    continue
                kept_total[ch] += int(keep.sum())
                awk = np.broadcast_to(aw, keep.shape)[keep]
                w2k = np.broadcast_to(W2, keep.shape)[keep]
                q2k = np.broadcast_to(iq2[None, None, :, None, None], keep.shape)[keep]
                q3k = np.broadcast_to(iq3[None, None, :, None, None], keep.shape)[keep]
                sp2 = np.broadcast_to(speed[iq2][None, None, :, :, None], keep.shape)[keep]
                win = 2.0 * sq * v_hi
                # sorted-scan threshold on the row frequency (and so on the lowest one at q'')
                thr = (w_hi - awk if s2 > 0 else awk - w_lo) + win
                slack = 1e-12 * (np.abs(awk) + w_hi + win)
                assert np.all(w2k <= thr + slack)
                assert np.all(wmin_q[q2k] <= thr + slack)
                # row cull: distance of x = aw s'' w'' from [w_min, w_max] of q'''
                x = awk + w2k if s2 > 0 else awk - w2k
                dist = np.maximum(np.maximum(x - wmax_q[q3k], wmin_q[q3k] - x), 0.0)
                lim = sq * (sp2 + vmax_q[q3k])
                assert np.all(dist <= lim * (1 + 1e-12) + 1e-12)
                # block cull: distance of 0 from the dw range of the block (q'', q''')
                if s2 > 0:
                    lo = awk + wmin_q[q2k] - wmax_q[q3k]
                    hi = awk + wmax_q[q2k] - wmin_q[q3k]
                else:
                    lo = awk - wmax_q[q2k] - wmax_q[q3k]
                    hi = awk - wmin_q[q2k] - wmin_q[q3k]
                bdist = np.maximum(np.maximum(lo, -hi), 0.0)
                blim = sq * (vmax_q[q2k] + vmax_q[q3k])
                assert np.all(bdist <= blim * (1 + 1e-12) + 1e-12)
    # the bounds were exercised on kept processes of both channels
    assert kept_total[0] > 0 and kept_total[2] > 0
