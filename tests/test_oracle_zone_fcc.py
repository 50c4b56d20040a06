"""Pins of the oracle's first-Brillouin-zone images and normal / Umklapp split on the FCC
(diamond-structure) cell, whose reciprocal basis is not orthogonal, and pins of the oracle's
partner-restricted sum.

The images are checked against what geometry fixes, by an independent search in numpy on
the synthetic crystal's reciprocal vectors (shifts -3..3, a wider range than the oracle's):

* k - q is a reciprocal-lattice vector (its reduced coordinates are integers);
* no image of q over the wider shift range is shorter than k (relative 1e-10);
* at the zone-boundary points of the 4x4x4 grid the number of equally short images and their
  length are the textbook values: L (2 images, |k| = sqrt(3) pi / a), X (2, 2 pi / a) and
  W (4, sqrt(5) pi / a);
* of equally short images the oracle keeps the first in the shift order m1, m2, m3 (m1
  slowest), the tie reading of the split (the paper does not print its representation of q).

The class counts of every kept process of sampled targets on the 4x4x4 diamond grid are then
recomputed by brute force: every candidate tested with the exact FP64 predicate and classed
with the numpy images (Q = k(q''') - (k(q) + s' k(q') + s'' k(q''))).
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from synth.crystal import grid_points, flat_index


def _numpy_images(cr, grid, span):
    """Every image q + G, G = sum_d m_d b_d, m_d in span: (points, shifts, vectors)."""
    B = np.asarray(cr.B)
    n = grid_points(grid)                                    # iq = n1 + g0 (n2 + g1 n3)
    f = n / np.asarray(grid, dtype=float)
    shifts = np.array(list(itertools.product(span, repeat=3)), dtype=float)
    vec = (f[:, None, :] + shifts[None, :, :]) @ B           # [iq][shift][3]
    return n, shifts, vec


@pytest.mark.parametrize("cell,grid", [("diamond", (4, 4, 4)), ("diamond", (3, 4, 5)),
                                       ("diamond", (6, 6, 6)), ("wurtzite", (6, 6, 4)),
                                       ("rhombohedral", (4, 4, 4))])
def test_first_zone_images(cell, grid):
    """The diamond cell's lattice matrix is symmetric; the hexagonal (wurtzite-like) and
    rhombohedral ones are not, so a transposed reciprocal basis fails there."""
    cr = {"diamond": synth.crystal.diamond, "wurtzite": synth.crystal.wurtzite_like,
          "rhombohedral": synth.crystal.layered_rhombohedral}[cell]()
    N = int(np.prod(grid))
    k = oracle.first_zone(cr.A, grid, np.arange(N))
    n, _, wide = _numpy_images(cr, grid, range(-3, 4))
    # k - q is a reciprocal-lattice vector: reduced coordinates k.a_d / 2 pi - n_d / N_d integer
    red = k @ np.asarray(cr.A).T / (2.0 * math.pi) - n / np.asarray(grid, dtype=float)
    assert np.max(np.abs(red - np.rint(red))) < 1e-12
    # no image over the wider range is shorter
    l2 = np.sum(k * k, axis=1)
    wmin = np.min(np.sum(wide * wide, axis=2), axis=1)
    assert np.all(l2 <= wmin * (1.0 + 1e-10) + 1e-30)
    # tie reading: the first shift (m1 slowest) among the equally short images in -2..1
    _, sh, vec = _numpy_images(cr, grid, range(-2, 2))
    vl2 = np.sum(vec * vec, axis=2)
    for iq in range(N):
        tied = np.nonzero(vl2[iq] <= vl2[iq].min() * (1.0 + 1e-10))[0]
        np.testing.assert_allclose(k[iq], vec[iq, tied[0]], rtol=0, atol=1e-12)


def test_zone_boundary_points_fcc():
    """L = b1/2, X = (b2 + b3)/2 and W = b1/4 + b2/2 + 3 b3/4 lie on the 4x4x4 grid."""
    cr = synth.crystal.diamond()
    a = 5.43
    grid = (4, 4, 4)
    cases = {"L": ((2, 0, 0), 2, math.sqrt(3.0) * math.pi / a),
             "X": ((0, 2, 2), 2, 2.0 * math.pi / a),
             "W": ((1, 2, 3), 4, math.sqrt(5.0) * math.pi / a)}
    _, _, wide = _numpy_images(cr, grid, range(-3, 4))
    for name, (nn, ntie, length) in cases.items():
        iq = int(flat_index(np.array(nn), grid))
        k = oracle.first_zone(cr.A, grid, [iq])[0]
        assert abs(np.linalg.norm(k) - length) < 1e-12 * length, name
        l2 = np.sum(wide[iq] * wide[iq], axis=1)
        assert np.count_nonzero(np.abs(l2 - length * length) < 1e-10 * length * length) == ntie, name


def test_class_counts_by_brute_force_fcc():
    """Normal / Umklapp counts of 6 targets on the 4x4x4 diamond grid (zone-boundary ties at
    L, X and W occur) against a brute-force classification with the numpy images."""
    inst = synth.diamond_instance((4, 4, 4), synth.configs.RC_FIRST, seed=12)
    grid = np.array(inst.grid)
    N, nb = inst.nq, inst.nb
    w = np.asarray(inst.omega, dtype=np.float64).reshape(N, nb)
    v = np.asarray(inst.vel, dtype=np.float64).reshape(N, nb, 3)
    act = w > 0
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    c_win = ((2.0 * 1.0) * dq) * ((2.0 * 1.0) * dq)
    n, sh, vec = _numpy_images(inst.cr, inst.grid, range(-2, 2))
    vl2 = np.sum(vec * vec, axis=2)
    img = np.zeros((N, 3), dtype=np.int64)                 # first-zone numerators n + m N
    for iq in range(N):
        tied = np.nonzero(vl2[iq] <= vl2[iq].min() * (1.0 + 1e-10))[0]
        img[iq] = n[iq] + sh[tied[0]].astype(np.int64) * grid
    flat = lambda m: m[..., 0] + grid[0] * (m[..., 1] + grid[1] * m[..., 2])
    tq = [1, 2, 21, 42, 27, 63]                            # includes the L, X and W points
    targets = np.array([iq * nb + j for iq in tq for j in range(nb)], dtype=np.int32)
    counts = np.zeros((len(targets), 3, 2), dtype=np.int64)
    for ch, (s1, s2) in enumerate([(1, 1), (1, -1), (-1, -1)]):
        for it, iq in enumerate(tq):
            for iq1 in range(N):
                iq2 = np.arange(N)
                iq3 = flat(np.mod(n[iq] + s1 * n[iq1] + s2 * n[iq2], grid))
                Q = img[iq3] - (img[iq] + s1 * img[iq1] + s2 * img[iq2])
                umk = np.any(Q != 0, axis=1)
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
                per_j = keep.sum(axis=(1, 3, 4))
                sl = slice(it * nb, (it + 1) * nb)
                counts[sl, ch, 0] += (per_j * ~umk[None, :]).sum(1)
                counts[sl, ch, 1] += (per_j * umk[None, :]).sum(1)
    m = oracle.Model.from_instance(inst)
    _, _, c = oracle.rates4(m, [300.0], 1.0, 7, dq, targets, want_rates=False)
    _, _, cn = oracle.rates4_class(m, inst.cr.A, 1, [300.0], 1.0, 7, dq, targets, want_rates=False)
    _, _, cu = oracle.rates4_class(m, inst.cr.A, 2, [300.0], 1.0, 7, dq, targets, want_rates=False)
    assert np.array_equal(counts[:, :, 0] + counts[:, :, 1], c)
    assert np.array_equal(counts[:, :, 0], cn)
    assert np.array_equal(counts[:, :, 1], cu)
    assert cn.sum() > 0 and cu.sum() > 0


def test_partner_sum_pins():
    """oracle_rates4_partners: with every q' listed it is the full sum (counts exact, rates to
    1e-13); disjoint q' lists covering the grid add up to it (counts exactly, rates 1e-13);
    the empty or out-of-range list is an error."""
    inst = synth.diamond_instance((3, 2, 2), synth.configs.RC_FIRST, seed=13, T=(300.0, 800.0))
    m = oracle.Model.from_instance(inst)
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    targets = np.arange(0, inst.nmodes, 5)
    r, _, c = oracle.rates4(m, inst.T, 1.0, 7, dq, targets)
    ra, ca = oracle.rates4_partners(m, inst.T, 1.0, 7, dq, targets, np.arange(inst.nq))
    assert np.array_equal(ca, c)
    np.testing.assert_allclose(ra, r, rtol=1e-13)
    rng = np.random.default_rng(3)
    perm = rng.permutation(inst.nq)
    parts = [perm[:4], perm[4:5], perm[5:]]
    rs, cs = zip(*(oracle.rates4_partners(m, inst.T, 1.0, 7, dq, targets, p) for p in parts))
    assert np.array_equal(sum(cs), c)
    assert all(x.sum() > 0 for x in cs)
    np.testing.assert_allclose(sum(rs), r, rtol=1e-13)
    with pytest.raises(ValueError):
        oracle.rates4_partners(m, inst.T, 1.0, 7, dq, targets, np.array([inst.nq]))
