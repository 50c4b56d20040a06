"""Pins of the oracle's normal / Umklapp split (the two process classes named after Eq. tao0:
Q = 0 is a normal process, Q != 0 an Umklapp one).

* The two classes partition the kept processes: rates add up to the unrestricted sum and
  counts add up exactly, for every channel.
* On a grid with the single point Gamma every process is normal.
* Brute force on a one-atom orthorhombic cell: with orthogonal reciprocal vectors the
  first-zone image of a grid point splits axis by axis, n_d / N_d or n_d / N_d - 1, the
  latter from n_d / N_d >= 1/2 on (the zone-boundary tie goes to the negative image, as the
  shift order -2..1 puts it first); a kept process is normal exactly when the images satisfy
  k(q) + s' k(q') + s'' k(q'') = k(q''') on every axis.  Every candidate is tested with the
  exact FP64 predicate and the per-target, per-channel class counts must equal the oracle's.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from synth import configs


def _split(inst, T, sb=1.0, mask=7):
    m = oracle.Model.from_instance(inst)
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    r, rc, c = oracle.rates4(m, T, sb, mask, dq)
    rn, rcn, cn = oracle.rates4_class(m, inst.cr.A, 1, T, sb, mask, dq)
    ru, rcu, cu = oracle.rates4_class(m, inst.cr.A, 2, T, sb, mask, dq)
    return (r, rc, c), (rn, rcn, cn), (ru, rcu, cu)


@pytest.mark.parametrize("which", ["small", "ortho"])
def test_normal_plus_umklapp_is_the_whole_sum(which):
    inst = synth.small() if which == "small" else configs.ortho()
    (r, rc, c), (rn, rcn, cn), (ru, rcu, cu) = _split(inst, [300.0, 900.0])
    assert np.array_equal(cn + cu, c)
    assert cn.sum() > 0 and cu.sum() > 0
    scale = np.maximum(np.abs(rc), 1e-300)
    assert np.max(np.abs(rcn + rcu - rc) / scale) < 1e-12
    assert np.max(np.abs(rn + ru - r) / np.maximum(np.abs(r), 1e-300)) < 1e-12


def test_gamma_only_grid_has_no_umklapp_process():
    rng = np.random.default_rng(9)
    C = rng.standard_normal((3, 3, 3, 3))
    C = sum(np.transpose(C, p) for p in itertools.permutations(range(4))) / 24.0
    w = np.array([[10.0, 20.0, 30.0]])
    evec = np.zeros((1, 3, 1, 3), dtype=complex)
    for j in range(3):
        evec[0, j, 0, j] = 1.0
    m = oracle.Model((1, 1, 1), [12.0], w, evec, np.zeros((1, 3, 3)),
                     np.zeros((1, 4), dtype=np.int32), np.zeros((1, 3, 3), dtype=np.int32),
                     C.reshape(1, 81))
    A = np.eye(3) * 3.0
    _, _, c = oracle.rates4(m, [400.0], 1.0, 7, 0.3)
    _, _, cn = oracle.rates4_class(m, A, 1, [400.0], 1.0, 7, 0.3)
    _, _, cu = oracle.rates4_class(m, A, 2, [400.0], 1.0, 7, 0.3)
    assert c.sum() > 0
    assert np.array_equal(cn, c) and cu.sum() == 0


def test_class_counts_by_brute_force_orthorhombic():
    inst = configs.ortho()
    grid = np.array(inst.grid)
    w = np.asarray(inst.omega, dtype=np.float64).reshape(-1, inst.nb)
    v = np.asarray(inst.vel, dtype=np.float64).reshape(-1, inst.nb, 3)
    N, nb = w.shape
    act = w > 0
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    c_win = ((2.0 * 1.0) * dq) * ((2.0 * 1.0) * dq)
    n = np.stack(np.meshgrid(*[np.arange(x) for x in grid], indexing="ij"), -1)
    n = n.transpose(2, 1, 0, 3).reshape(-1, 3)                    # iq = n1 + g0 (n2 + g1 n3)
    img = np.where(2 * n >= grid, n - grid, n)                    # first-zone numerators
    flat = lambda m: m[..., 0] + grid[0] * (m[..., 1] + grid[1] * m[..., 2])
    counts = np.zeros((N * nb, 3, 2), dtype=np.int64)             # [target][channel][N, U]
    for ch, (s1, s2) in enumerate([(1, 1), (1, -1), (-1, -1)]):
        for iq in range(N):
            for iq1 in range(N):
                iq2 = np.arange(N)
                iq3 = flat(np.mod(n[iq] + s1 * n[iq1] + s2 * n[iq2], grid))
                Q = img[iq3] - (img[iq] + s1 * img[iq1] + s2 * img[iq2])
                umk = np.any(Q != 0, axis=1)                          # per q''
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
                per_j = keep.sum(axis=(1, 3, 4))                       # [j][q'']
                counts[iq * nb:(iq + 1) * nb, ch, 0] += (per_j * ~umk[None, :]).sum(1)
                counts[iq * nb:(iq + 1) * nb, ch, 1] += (per_j * umk[None, :]).sum(1)
    (_, _, c), (_, _, cn), (_, _, cu) = _split(inst, [300.0])
    assert np.array_equal(counts[:, :, 0] + counts[:, :, 1], c)
    assert np.array_equal(counts[:, :, 0], cn)
    assert np.array_equal(counts[:, :, 1], cu)
    assert cn.sum() > 0 and cu.sum() > 0
