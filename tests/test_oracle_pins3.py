"""Pins of the FP64 three-phonon oracle (Eq. 3phgamma, Eq. V3) to facts that do not come
from the oracle itself.  The three-phonon rate is an input feature of the surrogate."""
import itertools
import math

import numpy as np
import pytest
import scipy.constants as sc

import oracle
import synth
from synth.crystal import grid_points, flat_index, minus_index
from synth.fc3 import FC3, random_fc3
from tests import brute
from tests.test_oracle_pins import _rotate_q, _degenerate_sums

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _dq(inst):
    return oracle.default_dq(inst.cr.A, inst.grid)


@pytest.fixture(scope="module")
def inst3():
    inst = synth.diamond_instance((3, 3, 3), synth.configs.RC_FIRST, seed=21)
    fc3 = random_fc3(inst.cr, 3.0, np.random.default_rng(21))
    return inst, fc3, oracle.Model.from_instance(inst)


@pytest.fixture(scope="module")
def inst4():
    inst = synth.diamond_instance((4, 4, 4), synth.configs.RC_FIRST, seed=22)
    fc3 = random_fc3(inst.cr, 4.0, np.random.default_rng(22))
    return inst, fc3, oracle.Model.from_instance(inst)


def test_c3_against_codata():
    """The Eq. 3phgamma prefactor hbar pi / 4 in the library's units, against scipy's
    CODATA constants (catches a wrong power of ten, a missing sqrt of the mass unit)."""
    kv = sc.electron_volt / (sc.angstrom**3 * sc.atomic_mass**1.5)
    ref = sc.hbar * math.pi / 4 * kv**2 * 1e-60
    assert oracle.c3() == pytest.approx(ref, rel=2e-8)
    assert oracle.c3() == pytest.approx(brute.c3_si(), rel=1e-14)


def _momentum_triples(inst, rng, n):
    grid = np.asarray(inst.grid)
    pts = grid_points(inst.grid)
    out_m, out_s = [], []
    while len(out_m) < n:
        sg = rng.choice([-1, 1], size=3)
        sg[0] = 1
        iq = rng.integers(0, inst.nq, size=2)
        n3 = -(sg[0] * pts[iq[0]] + sg[1] * pts[iq[1]]) * sg[2]
        iq3 = int(flat_index(n3 % grid, inst.grid))
        js = rng.integers(0, inst.nb, size=3)
        modes = [int(iq[0]) * inst.nb + js[0], int(iq[1]) * inst.nb + js[1], iq3 * inst.nb + js[2]]
        if min(inst.omega.reshape(-1)[modes]) <= 0:
            continue
        out_m.append(modes)
        out_s.append(list(sg))
    return np.array(out_m), np.array(out_s)


def _scale3(inst, fc3, modes):
    ev = inst.evec.reshape(inst.nmodes, inst.cr.natoms, 3)
    sq = np.sqrt(inst.cr.mass)
    tot = 0.0
    absphi = np.abs(fc3.phi).reshape(-1, 3, 3, 3)
    for n in range(fc3.n):
        X = [np.abs(ev[modes[s], fc3.atoms[n, s]]) / sq[fc3.atoms[n, s]] for s in range(3)]
        tot += np.einsum("abc,a,b,c->", absphi[n], *X)
    return tot


def test_v3_permutation_invariance(inst4):
    """V (Eq. V3) is invariant under the 6 permutations of its (mode, sign) slots for
    momentum-conserving triples, Umklapp included (catches a conjugation on the wrong slot,
    a phase on the wrong cell, swapped Cartesian indices)."""
    inst, fc3, m = inst4
    modes, signs = _momentum_triples(inst, np.random.default_rng(31), 8)
    nontrivial = 0
    for i in range(len(modes)):
        perms = list(itertools.permutations(range(3)))
        V = oracle.v3(m, fc3, np.array([modes[i][list(p)] for p in perms]),
                      np.array([signs[i][list(p)] for p in perms]))
        scale = _scale3(inst, fc3, modes[i])
        assert np.max(np.abs(V - V[0])) <= 1e-12 * scale
        nontrivial += abs(V[0]) > 1e-6 * scale     # some elements vanish by symmetry
    assert nontrivial >= len(modes) // 2


def test_v3_time_reversal(inst4):
    """(q, j) -> (-q, j) in every slot with every sign flipped leaves V unchanged."""
    inst, fc3, m = inst4
    modes, signs = _momentum_triples(inst, np.random.default_rng(32), 8)
    mq = minus_index(inst.grid)
    tr = mq[modes // inst.nb] * inst.nb + modes % inst.nb
    np.testing.assert_allclose(oracle.v3(m, fc3, tr, -signs), oracle.v3(m, fc3, modes, signs),
                               rtol=1e-13)


def test_v3_acoustic_sum_rule(inst4):
    """With any slot a Gamma acoustic mode V vanishes (acoustic sum rule on Phi and a rigid
    translation eigenvector)."""
    inst, fc3, m = inst4
    modes, signs = _momentum_triples(inst, np.random.default_rng(33), 6)
    pts = grid_points(inst.grid)
    for i in range(len(modes)):
        for slot in range(3):
            for ac in range(3):
                md, sg = modes[i].copy(), signs[i].copy()
                other = (slot + 1) % 3
                qs = [pts[x // inst.nb] * s for x, s in zip(md, sg)]
                newq = (qs[other] + qs[slot]) * sg[other] % np.asarray(inst.grid)
                md[other] = int(flat_index(newq, inst.grid)) * inst.nb + md[other] % inst.nb
                md[slot] = ac
                if min(inst.omega.reshape(-1)[md[[s for s in range(3) if s != slot]]]) <= 0:
                    continue
                V = oracle.v3(m, fc3, md[None, :], sg[None, :])[0]
                assert abs(V) <= 1e-12 * _scale3(inst, fc3, md)


def test_v3_closed_form_single_component():
    """One triplet with one non-zero component on a 2x1x1 grid: V is the product of three
    eigenvector components, 1/sqrt(M M M) and the phase exp(i pi n R)."""
    grid = (2, 1, 1)
    rng = np.random.default_rng(4)
    mass = np.array([7.0, 56.0])
    omega = np.full((2, 6), 10.0)
    evec = rng.standard_normal((2, 6, 2, 3)) + 1j * rng.standard_normal((2, 6, 2, 3))
    vel = np.zeros((2, 6, 3))
    m = oracle.Model(grid, mass, omega, evec, vel, np.zeros((1, 4), np.int32),
                     np.zeros((1, 3, 3), np.int32), np.zeros((1, 81)))
    phi = np.zeros((1, 27))
    phi[0, (2 * 3 + 0) * 3 + 1] = 3.5
    fc3 = FC3(np.array([[0, 1, 1]], np.int32), np.array([[[1, 0, 0], [0, 0, 0]]], np.int32), phi)
    # (q=1,j=2) (q=1,j=0) (q=0,j=5); signs + - -:  1 - 1 - 0 = 0
    V = oracle.v3(m, fc3, np.array([[8, 6, 5]]), np.array([[1, -1, -1]]))[0]
    e = evec.reshape(12, 2, 3)
    ref = 3.5 * e[8, 0, 2] * np.conj(e[6, 1, 0] * np.exp(1j * np.pi)) * np.conj(e[5, 1, 1])
    assert V == pytest.approx(ref / math.sqrt(7.0 * 56.0 * 56.0), rel=1e-14)


def test_rates3_closed_form_gamma_only():
    """One atom, N = 1, branches 10/20/30 rad/ps along x/y/z, zero velocities and one
    on-site symmetric tensor: the rate is a hand-enumerable sum with the (n' - n'') and
    (n' + n'' + 1)/2 occupation forms (catches the channel weight, a swapped occupation,
    the 1/(w w' w'') factor or the prefactor)."""
    rng = np.random.default_rng(10)
    C = rng.standard_normal((3, 3, 3))
    C = sum(np.transpose(C, p) for p in itertools.permutations(range(3))) / 6.0
    M = 12.0
    w = np.array([10.0, 20.0, 30.0])
    evec = np.zeros((1, 3, 1, 3), dtype=complex)
    for j in range(3):
        evec[0, j, 0, j] = 1.0
    m = oracle.Model((1, 1, 1), [M], w[None, :], evec, np.zeros((1, 3, 3)),
                     np.zeros((1, 4), np.int32), np.zeros((1, 3, 3), np.int32), np.zeros((1, 81)))
    fc3 = FC3(np.zeros((1, 3), np.int32), np.zeros((1, 2, 3), np.int32), C.reshape(1, 27))
    T = 400.0
    r, cnt = oracle.rates3(m, fc3, [T], 1.0, 0.3)
    n = 1.0 / np.expm1(sc.hbar / sc.k * 1e12 * w / T)
    kv = sc.electron_volt / (sc.angstrom**3 * sc.atomic_mass**1.5)
    pref = sc.hbar * math.pi / 4 * kv**2 * 1e-60
    for j in range(3):
        tot = 0.0
        for a, b in itertools.product(range(3), repeat=2):
            V2 = C[j, a, b] ** 2 / M**3
            wp = w[j] * w[a] * w[b]
            if w[j] + w[a] == w[b]:
                tot += pref * (n[a] - n[b]) * V2 / wp
            if w[j] == w[a] + w[b]:
                tot += 0.5 * pref * (n[a] + n[b] + 1) * V2 / wp
        assert r[0, j] == pytest.approx(tot, rel=2e-8)
    assert list(cnt[:, 0]) == [2, 1, 0] and list(cnt[:, 1]) == [0, 1, 2]


def test_rates3_brute_force(inst3):
    """Full 3x3x3 rates against the double-loop brute force with an explicit momentum
    Kronecker delta: identical kept counts, rates to rounding."""
    inst, fc3, m = inst3
    dq = _dq(inst)
    targets = np.arange(0, inst.nmodes, 5)
    r, c = oracle.rates3(m, fc3, [300.0, 800.0], 1.0, dq, targets)
    rb, cb = brute.brute_rates3(inst.grid, inst.cr.mass, inst.omega, inst.evec, inst.vel,
                                fc3.atoms, fc3.cells, fc3.phi, [300.0, 800.0], 1.0, dq, targets)
    assert np.array_equal(c, cb)
    assert c.sum() > 100
    np.testing.assert_allclose(r, rb, rtol=1e-11, atol=1e-300)


def test_rates3_time_reversal(inst3):
    inst, fc3, m = inst3
    mq = minus_index(inst.grid)
    qs = [1, 5, 14]
    t1 = [q * inst.nb + j for q in qs for j in range(inst.nb)]
    t2 = [mq[q] * inst.nb + j for q in qs for j in range(inst.nb)]
    r1, c1 = oracle.rates3(m, fc3, [300.0], 1.0, _dq(inst), t1)
    r2, c2 = oracle.rates3(m, fc3, [300.0], 1.0, _dq(inst), t2)
    assert np.array_equal(c1, c2)
    np.testing.assert_allclose(r1, r2, rtol=1e-13)


def test_rates3_symmetry_equivalent_q(inst4):
    """Degenerate-set sums of the rate agree at q and its space-group images (space-group
    covariant FC3 and harmonic model)."""
    inst, fc3, m = inst4
    rng = np.random.default_rng(6)
    ops = [inst.cr.ops[i] for i in rng.choice(len(inst.cr.ops), size=4, replace=False)]
    iq0 = 6
    qs = [iq0] + [_rotate_q(inst, T, iq0) for (T, t) in ops]
    assert len(set(qs)) > 1
    targets = [q * inst.nb + j for q in qs for j in range(inst.nb)]
    r, _ = oracle.rates3(m, fc3, [300.0], 1.0, _dq(inst), targets)
    r = r.reshape(len(qs), inst.nb)
    sums = np.array([_degenerate_sums(inst.omega[q], r[k]) for k, q in enumerate(qs)])
    for k in range(1, len(qs)):
        np.testing.assert_allclose(sums[k], sums[0], rtol=1e-10)


def test_rates3_scaling(inst3):
    """Doubling Phi multiplies every rate by exactly 4; in the classical limit every
    occupation form of Eq. 3phgamma grows as T (catches a squared occupation)."""
    inst, fc3, m = inst3
    dq = _dq(inst)
    targets = np.arange(3, inst.nmodes, 7)
    r, c = oracle.rates3(m, fc3, [1e6, 2e6], 1.0, dq, targets)
    np.testing.assert_allclose(r[1] / r[0], 2.0, rtol=2e-3)
    f2 = FC3(fc3.atoms, fc3.cells, 2.0 * fc3.phi)
    r2, c2 = oracle.rates3(m, f2, [1e6, 2e6], 1.0, dq, targets)
    assert np.array_equal(c2, c) and np.array_equal(r2, 4.0 * r)
