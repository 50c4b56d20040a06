"""Pins of the oracle's four-phonon phase spaces (P4 and the weighted WP4: the rate sum of
Eq. tao0 with |V|^2 and the prefactor of Eq. 4phgamma set to 1).

* Flat bands with zero group velocity: every kept process has dw = 0 exactly and sigma = 0,
  so delta is the clamp value 1 and both sums have closed forms: P4 = sum_s c_s n_s / N^2
  from the kept-process counts n_s, and WP4 the occupation factors over the frequency
  products of the kept processes, enumerated here by brute force.
* The phase spaces do not depend on the force constants, P4 not on temperature, and the
  kept-process counts equal those of the rate sum.
"""
import itertools

import numpy as np

import oracle
import synth

HK = 6.62607015e-34 / (2.0 * np.pi * 1.380649e-23) * 1e12   # hbar / k_B in K ps (SI 2019 h, k_B)


def _flat(nq_grid=(2, 2, 2)):
    rng = np.random.default_rng(11)
    C = rng.standard_normal((3, 3, 3, 3))
    C = sum(np.transpose(C, p) for p in itertools.permutations(range(4))) / 24.0
    nq = int(np.prod(nq_grid))
    w = np.tile(np.array([10.0, 20.0, 30.0]), (nq, 1))
    evec = np.zeros((nq, 3, 1, 3), dtype=complex)
    for j in range(3):
        evec[:, j, 0, j] = 1.0
    return oracle.Model(nq_grid, [12.0], w, evec, np.zeros((nq, 3, 3)),
                        np.zeros((1, 4), dtype=np.int32), np.zeros((1, 3, 3), dtype=np.int32),
                        C.reshape(1, 81)), w


def test_flat_bands_closed_forms():
    m, w = _flat()
    T = [300.0, 900.0]
    nq = w.shape[0]
    P4, P4ch, c = oracle.phase_space4(m, 2, T, 1.0, 7, 0.3)
    WP4, _, c2 = oracle.phase_space4(m, 1, T, 1.0, 7, 0.3)
    assert np.array_equal(c, c2) and c.sum() > 0
    cw = np.array([0.5, 0.5, 1.0 / 6.0])
    # P4: every kept process contributes delta = 1
    expect = (c * cw[None, :]).sum(1) / nq**2
    for t in range(len(T)):
        assert np.allclose(P4[t], expect, rtol=1e-14, atol=0.0)
    # WP4 by brute force: all q coincide in frequency, so the kept set is the set of branch
    # quadruples with exact frequency balance, repeated for every (q', q'')
    wb = w[0]
    for t, TT in enumerate(T):
        n0 = 1.0 / np.expm1(HK * wb / TT)
        for j in range(3):
            tot = 0.0
            for ch, (s1, s2) in enumerate([(1, 1), (1, -1), (-1, -1)]):
                for j1, j2, j3 in itertools.product(range(3), repeat=3):
                    if ((wb[j] + s1 * wb[j1]) + s2 * wb[j2]) - wb[j3] != 0.0:
                        continue
                    if ch == 0:
                        f = (1 + n0[j1]) * (1 + n0[j2]) * n0[j3] / n0[j]
                    elif ch == 1:
                        f = (1 + n0[j1]) * n0[j2] * n0[j3] / n0[j]
                    else:
                        f = n0[j1] * n0[j2] * n0[j3] / n0[j]
                    tot += cw[ch] * f / (wb[j] * wb[j1] * wb[j2] * wb[j3]) * nq * nq
            for iq in range(nq):
                assert np.isclose(WP4[t, iq * 3 + j], tot / nq**2, rtol=1e-12, atol=0.0)


def test_force_constant_and_temperature_independence():
    inst = synth.small()
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    targets = np.arange(0, inst.nmodes, 7)
    m1 = oracle.Model.from_instance(inst)
    m2 = oracle.Model.from_instance(inst, phi_scale=2.0)
    T = [200.0, 800.0]
    for kind in (1, 2):
        a, _, ca = oracle.phase_space4(m1, kind, T, 1.0, 7, dq, targets)
        b, _, cb = oracle.phase_space4(m2, kind, T, 1.0, 7, dq, targets)
        assert np.array_equal(a, b) and np.array_equal(ca, cb)
    p4, _, _ = oracle.phase_space4(m1, 2, T, 1.0, 7, dq, targets)
    assert np.array_equal(p4[0], p4[1]) and p4.max() > 0
    _, _, c = oracle.rates4(m1, T, 1.0, 7, dq, targets, want_rates=False)
    assert np.array_equal(ca, c)
