"""Pins of the FP64 oracle to facts that do not come from the oracle itself.

Each test names what it pins and which plausible mistake it would catch.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.constants as sc
from scipy import integrate

import oracle
import synth
from synth.crystal import grid_points, flat_index, minus_index
from synth.fc4 import FC4, random_fc4
from tests import brute

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


@pytest.fixture(scope="module")
def small():
    return synth.small()


@pytest.fixture(scope="module")
def small_model(small):
    return oracle.Model.from_instance(small)


def _dq(inst):
    return oracle.default_dq(inst.cr.A, inst.grid)


# ------------------------------------------------------------------------- constants

def test_constants_against_codata():
    """hbar/k_B and the Eq. 4phgamma prefactor against scipy's CODATA values
    (catches a wrong power of ten or unit in C4)."""
    hk = sc.hbar / sc.k * 1e12
    assert oracle.hbar_over_kb() == pytest.approx(hk, rel=1e-9)
    kv = sc.electron_volt / (sc.angstrom**4 * sc.atomic_mass**2)
    # Gamma[1/s] = hbar^2 pi/8 (V kv)^2 delta[s] / omega[1/s]^4 ; convert to ps units
    c4 = sc.hbar**2 * math.pi / 8 * kv**2 * 1e-12 * 1e-12 / 1e48
    # the oracle types CODATA 2018 values; scipy may carry a later CODATA set (the atomic
    # mass unit moved by 1.4e-9 relative between them, and C4 goes as amu^-4)
    assert oracle.c4() == pytest.approx(c4, rel=2e-8)


def test_bose_limits():
    """n0 = 1/(exp(x)-1): classical series kT/(hbar w) - 1/2 + x/12 for small x and
    exp(-x) for large x (catches exp vs expm1 or a missing hbar/k_B factor)."""
    hk = sc.hbar / sc.k * 1e12
    T = 300.0
    for w in (1e-4, 1e-2):
        x = hk * w / T
        assert oracle.bose(w, T) == pytest.approx(1 / x - 0.5 + x / 12, rel=1e-10)
    w = 500.0
    x = hk * w / T
    assert oracle.bose(w, T) == pytest.approx(math.exp(-x), rel=1e-5)


def test_delta_normalisation_and_window():
    """The adaptive Gaussian integrates to 1 and the |dw| <= 2 sigma window holds
    erf(2) of its weight (Sec. 2.4); the small-sigma branch returns 1."""
    sigma = 0.37
    tot, _ = integrate.quad(lambda x: oracle.delta(x, sigma**2), -20 * sigma, 20 * sigma,
                            limit=200)
    assert tot == pytest.approx(1.0, rel=1e-10)
    win, _ = integrate.quad(lambda x: oracle.delta(x, sigma**2), -2 * sigma, 2 * sigma)
    assert win == pytest.approx(math.erf(2.0), rel=1e-10)
    assert oracle.delta(0.3, (0.5e-4) ** 2, 1e-4) == 1.0
    assert oracle.delta(0.0, (2e-4) ** 2, 1e-4) == pytest.approx(1 / (math.sqrt(math.pi) * 2e-4))


def test_default_dq():
    """Cube root of the reciprocal-cell volume per grid point; equals |b|/N-like spacing
    2 pi / (a N) * 4^(1/3)... checked against the direct determinant."""
    cr = synth.diamond()
    for grid in [(3, 3, 3), (8, 8, 8), (4, 3, 2)]:
        B = cr.B
        ref = (abs(np.linalg.det(B)) / np.prod(grid)) ** (1 / 3)
        assert oracle.default_dq(cr.A, grid) == pytest.approx(ref, rel=1e-14)


# ------------------------------------------------------------------------- enumeration

@pytest.mark.parametrize("grid", [(2, 2, 2), (3, 2, 1)])
def test_brute_force_momentum_delta(grid):
    """Oracle (folded q''') against an explicit Kronecker delta over every q''' with a
    literal einsum V: identical kept-process counts, rates to 1e-12 (catches a wrong fold,
    a wrong channel sign, a dropped channel weight or a transposed slot)."""
    inst = synth.diamond_instance(grid, synth.configs.RC_FIRST, seed=5, T=(300.0, 900.0))
    m = oracle.Model.from_instance(inst)
    dq = _dq(inst)
    targets = np.arange(inst.nmodes)
    r_o, _, c_o = oracle.rates4(m, inst.T, 1.0, 7, dq, targets)
    r_b, c_b = brute.brute_rates(inst.grid, inst.cr.mass, inst.omega, inst.evec, inst.vel,
                                 inst.fc4.atoms, inst.fc4.cells, inst.fc4.phi, inst.T, 1.0, 7,
                                 dq, targets)
    assert np.array_equal(c_o, c_b)
    assert c_o.sum() > 0
    np.testing.assert_allclose(r_o, r_b, rtol=1e-12, atol=1e-300)


def test_brute_force_second_shell_sampled():
    """Same check with the second-shell FC4 (1522 quartets), sampled targets."""
    inst = synth.diamond_instance((2, 2, 2), synth.configs.RC_SECOND, seed=6, T=(500.0,))
    m = oracle.Model.from_instance(inst)
    dq = _dq(inst)
    targets = np.array([3, 7, 11, 40, 47])
    r_o, _, c_o = oracle.rates4(m, inst.T, 0.7, 7, dq, targets)
    r_b, c_b = brute.brute_rates(inst.grid, inst.cr.mass, inst.omega, inst.evec, inst.vel,
                                 inst.fc4.atoms, inst.fc4.cells, inst.fc4.phi, inst.T, 0.7, 7,
                                 dq, targets)
    assert np.array_equal(c_o, c_b)
    np.testing.assert_allclose(r_o, r_b, rtol=1e-12)


# ------------------------------------------------------------------------- matrix element

def _momentum_quads(inst, rng, n, umklapp=True):
    """Random (mode, sign) quadruples with s1 q1 + s2 q2 + s3 q3 + s4 q4 = 0 mod grid."""
    grid = np.asarray(inst.grid)
    pts = grid_points(inst.grid)
    out_m, out_s = [], []
    while len(out_m) < n:
        sg = rng.choice([-1, 1], size=4)
        sg[0] = 1
        iq = rng.integers(0, inst.nq, size=3)
        n4 = -(sg[0] * pts[iq[0]] + sg[1] * pts[iq[1]] + sg[2] * pts[iq[2]]) * sg[3]
        iq4 = int(flat_index(n4 % grid, inst.grid))
        tot = sg[0] * pts[iq[0]] + sg[1] * pts[iq[1]] + sg[2] * pts[iq[2]] + sg[3] * pts[iq4]
        if not umklapp and np.any(tot != 0):
            continue
        js = rng.integers(0, inst.nb, size=4)
        modes = [int(iq[0]) * inst.nb + js[0], int(iq[1]) * inst.nb + js[1],
                 int(iq[2]) * inst.nb + js[2], iq4 * inst.nb + js[3]]
        if min(inst.omega.reshape(-1)[modes]) <= 0:
            continue
        out_m.append(modes)
        out_s.append(list(sg))
    return np.array(out_m), np.array(out_s)


def _term_scale(inst, modes):
    """sum over quartets and components of |Phi| |X1||X2||X3||X4| (rounding scale of V)."""
    ev = inst.evec.reshape(inst.nmodes, inst.cr.natoms, 3)
    sq = np.sqrt(inst.cr.mass)
    tot = 0.0
    absphi = np.abs(inst.fc4.phi).reshape(-1, 3, 3, 3, 3)
    for n in range(inst.fc4.n):
        X = [np.abs(ev[modes[s], inst.fc4.atoms[n, s]]) / sq[inst.fc4.atoms[n, s]] for s in range(4)]
        tot += np.einsum("abcd,a,b,c,d->", absphi[n], *X)
    return tot


@pytest.fixture(scope="module")
def inst44():
    return synth.diamond_instance((4, 4, 4), synth.configs.RC_SECOND, seed=7)


def test_v4_permutation_invariance(inst44):
    """V (Eq. V4) is invariant under the 24 permutations of its four (mode, sign) slots for
    momentum-conserving quadruples, Umklapp included (P:Eq. TS symmetry of Phi).  Catches a
    conjugation on the wrong slot, a phase with the wrong sign or cell, a swapped
    Cartesian index."""
    m = oracle.Model.from_instance(inst44)
    rng = np.random.default_rng(11)
    modes, signs = _momentum_quads(inst44, rng, 6)
    for i in range(len(modes)):
        pm, ps = [], []
        for p in itertools.permutations(range(4)):
            pm.append(modes[i][list(p)])
            ps.append(signs[i][list(p)])
        V = oracle.v4(m, np.array(pm), np.array(ps))
        scale = _term_scale(inst44, modes[i])
        assert np.max(np.abs(V - V[0])) <= 1e-12 * scale
        assert abs(V[0]) > 1e-6 * scale   # non-trivial


def test_v4_time_reversal(inst44):
    """Replacing every mode by its time-reversed partner (-q, j) and flipping every slot
    sign leaves V unchanged (e(-q) = conj e(q) and the conjugate-symmetric phase table)."""
    m = oracle.Model.from_instance(inst44)
    rng = np.random.default_rng(12)
    modes, signs = _momentum_quads(inst44, rng, 8)
    mq = minus_index(inst44.grid)
    tr = (mq[modes // inst44.nb]) * inst44.nb + modes % inst44.nb
    V = oracle.v4(m, modes, signs)
    Vt = oracle.v4(m, tr, -signs)
    np.testing.assert_allclose(Vt, V, rtol=1e-13, atol=1e-300)


def test_v4_acoustic_sum_rule(inst44):
    """With any slot a Gamma acoustic mode, V vanishes (Eq. ASR): the sum over the atom of
    that slot of Phi is zero and the acoustic eigenvector is a rigid translation."""
    m = oracle.Model.from_instance(inst44)
    rng = np.random.default_rng(13)
    modes, signs = _momentum_quads(inst44, rng, 6)
    for i in range(len(modes)):
        for slot in range(4):
            for ac in range(3):
                md = modes[i].copy()
                sg = signs[i].copy()
                # put Gamma acoustic branch `ac` into `slot`; keep momentum: move the
                # removed momentum into the next slot
                other = (slot + 1) % 4
                pts = grid_points(inst44.grid)
                qs = [pts[x // inst44.nb] * s for x, s in zip(md, sg)]
                rem = qs[slot]
                newq = (qs[other] + rem) * sg[other] % np.asarray(inst44.grid)
                md[other] = int(flat_index(newq, inst44.grid)) * inst44.nb + md[other] % inst44.nb
                md[slot] = ac
                V = oracle.v4(m, md[None, :], sg[None, :])[0]
                if min(inst44.omega.reshape(-1)[md[[s for s in range(4) if s != slot]]]) <= 0:
                    continue
                scale = _term_scale(inst44, md)
                assert abs(V) <= 1e-12 * scale


def test_v4_closed_form_single_component():
    """One quartet with one non-zero component on a 2x1x1 grid: V is the product of the
    four eigenvector components, masses and the lattice phase exp(i pi n R) (catches a
    wrong mass power, a missing phase or a conjugation error)."""
    grid = (2, 1, 1)
    nat = 2
    rng = np.random.default_rng(3)
    mass = np.array([7.0, 56.0])
    omega = np.full((2, 6), 10.0)
    evec = rng.standard_normal((2, 6, nat, 3)) + 1j * rng.standard_normal((2, 6, nat, 3))
    vel = np.zeros((2, 6, 3))
    atoms = np.array([[0, 1, 1, 0]], dtype=np.int32)
    cells = np.array([[[1, 0, 0], [0, 0, 0], [1, 0, 0]]], dtype=np.int32)
    comp = (2 * 3 + 0) * 9 + 1 * 3 + 2   # alpha=2, beta=0, gamma=1, theta=2
    phi = np.zeros((1, 81))
    phi[0, comp] = 3.5
    m = oracle.Model(grid, mass, omega, evec, vel, atoms, cells, phi)
    # modes: (q=1,j=2) (q=1,j=0) (q=0,j=5) (q=0,j=3); signs + - + -:  1 - 1 + 0 - 0 = 0
    modes = np.array([[1 * 6 + 2, 1 * 6 + 0, 0 * 6 + 5, 0 * 6 + 3]])
    signs = np.array([[1, -1, 1, -1]])
    V = oracle.v4(m, modes, signs)[0]
    e = evec.reshape(12, nat, 3)
    ph_j = np.exp(1j * np.pi * 1 * 1)     # q=1 (n=1 of 2) on R_j = (1,0,0): exp(i pi) = -1
    ref = 3.5 * e[8, 0, 2] * np.conj(e[6, 1, 0] * ph_j) * e[5, 1, 1] * np.conj(e[3, 0, 2])
    ref /= math.sqrt(7.0 * 56.0 * 56.0 * 7.0)
    assert V == pytest.approx(ref, rel=1e-14)


# ------------------------------------------------------------------------- rates

def test_rates_closed_form_gamma_only():
    """A one-atom crystal sampled only at Gamma (N = 1), branches along x, y, z with
    frequencies 10, 20, 30 rad/ps, zero velocities (so only exactly energy-conserving
    processes survive and delta = 1 by the small-sigma rule) and a single on-site quartet
    with a fully symmetric random tensor.  The rate of each branch is then a finite
    hand-enumerable sum (catches wrong occupation forms, channel weights 1/2, 1/2, 1/6,
    the 1/(w w' w'' w''') factor or the prefactor)."""
    rng = np.random.default_rng(9)
    C = rng.standard_normal((3, 3, 3, 3))
    C = sum(np.transpose(C, p) for p in itertools.permutations(range(4))) / 24.0
    M = 12.0
    w = np.array([10.0, 20.0, 30.0])
    evec = np.zeros((1, 3, 1, 3), dtype=complex)
    for j in range(3):
        evec[0, j, 0, j] = 1.0
    m = oracle.Model((1, 1, 1), [M], w[None, :], evec, np.zeros((1, 3, 3)),
                     np.zeros((1, 4), dtype=np.int32), np.zeros((1, 3, 3), dtype=np.int32),
                     C.reshape(1, 81))
    T = 400.0
    r, rch, cnt = oracle.rates4(m, [T], 1.0, 7, 0.3)
    hk = sc.hbar / sc.k * 1e12
    n = 1.0 / np.expm1(hk * w / T)
    kv = sc.electron_volt / (sc.angstrom**4 * sc.atomic_mass**2)
    pref = sc.hbar**2 * math.pi / 8 * kv**2 * 1e-72
    for j in range(3):
        tot = 0.0
        for a, b, c in itertools.product(range(3), repeat=3):
            V2 = (C[j, a, b, c] / M**2) ** 2
            wp = w[j] * w[a] * w[b] * w[c]
            if w[j] + w[a] + w[b] == w[c]:
                tot += 0.5 * pref * (1 + n[a]) * (1 + n[b]) * n[c] / n[j] * V2 / wp
            if w[j] + w[a] == w[b] + w[c]:
                tot += 0.5 * pref * (1 + n[a]) * n[b] * n[c] / n[j] * V2 / wp
            if w[j] == w[a] + w[b] + w[c]:
                tot += pref / 6 * n[a] * n[b] * n[c] / n[j] * V2 / wp
        # prefactor from scipy's CODATA set (amu differs from CODATA 2018 by 1.4e-9)
        assert r[0, j] == pytest.approx(tot, rel=2e-8)


def test_rates_time_reversal(small, small_model):
    """rate(q, j) = rate(-q, j): the mirrored process set has bit-identical predicates, so
    counts are equal and rates agree up to summation order."""
    mq = minus_index(small.grid)
    qs = [1, 4, 13, 22]
    targets = [q * small.nb + j for q in qs for j in range(small.nb)]
    mirror = [mq[q] * small.nb + j for q in qs for j in range(small.nb)]
    r1, _, c1 = oracle.rates4(small_model, [300.0], 1.0, 7, _dq(small), targets)
    r2, _, c2 = oracle.rates4(small_model, [300.0], 1.0, 7, _dq(small), mirror)
    assert np.array_equal(c1, c2)
    np.testing.assert_allclose(r1, r2, rtol=1e-13)


def _rotate_q(inst, T, iq):
    cr = inst.cr
    n = grid_points(inst.grid)[iq] / np.asarray(inst.grid, float)
    qc = n @ cr.B
    f = (T @ qc) @ cr.A.T / (2 * np.pi) * np.asarray(inst.grid)
    fi = np.rint(f)
    assert np.max(np.abs(f - fi)) < 1e-9
    return int(flat_index(fi.astype(int) % np.asarray(inst.grid), inst.grid))


def _degenerate_sums(omega_q, r):
    w = omega_q
    tol = 1e-6 * max(1.0, w.max())
    out, cur = [], [0]
    for j in range(1, len(w)):
        if abs(w[j] - w[cur[-1]]) <= tol:
            cur.append(j)
        else:
            out.append(cur)
            cur = [j]
    out.append(cur)
    return np.array([r[..., s].sum(axis=-1) for s in out]).T


@pytest.mark.parametrize("rc", [synth.configs.RC_FIRST, synth.configs.RC_SECOND])
def test_rates_symmetry_equivalent_q(rc):
    """Rates summed over degenerate sets are equal at q and at its images under the
    space-group rotations (requires the Fd-3m-symmetric harmonic model and FC4, Eq. SGSO)."""
    grid = (3, 3, 3) if rc == synth.configs.RC_FIRST else (2, 2, 2)
    inst = synth.diamond_instance(grid, rc, seed=8)
    m = oracle.Model.from_instance(inst)
    dq = _dq(inst)
    iq0 = 1
    rng = np.random.default_rng(5)
    ops = [inst.cr.ops[i] for i in rng.choice(len(inst.cr.ops), size=4, replace=False)]
    qs = [iq0] + [_rotate_q(inst, T, iq0) for (T, t) in ops]
    assert len(set(qs)) > 1
    targets = [q * inst.nb + j for q in qs for j in range(inst.nb)]
    r, _, c = oracle.rates4(m, [300.0], 1.0, 7, dq, targets)
    r = r.reshape(len(qs), inst.nb)
    sums = np.array([_degenerate_sums(inst.omega[q], r[k]) for k, q in enumerate(qs)])
    for k in range(1, len(qs)):
        np.testing.assert_allclose(sums[k], sums[0], rtol=1e-10)


def test_rates_mask_additivity_and_phi_scaling(small, small_model):
    """Channel masks add up; doubling Phi multiplies every rate by exactly 4 with identical
    counts (V is linear in Phi and the arithmetic scales by powers of two exactly)."""
    dq = _dq(small)
    targets = np.arange(0, small.nmodes, 17)
    r7, rch, c7 = oracle.rates4(small_model, [300.0], 1.0, 7, dq, targets)
    parts = [oracle.rates4(small_model, [300.0], 1.0, 1 << ch, dq, targets) for ch in range(3)]
    np.testing.assert_allclose(sum(p[0] for p in parts), r7, rtol=1e-13)
    for ch in range(3):
        assert np.array_equal(parts[ch][2][:, ch], c7[:, ch])
        np.testing.assert_allclose(parts[ch][0][0], rch[0, ch], rtol=1e-13)
    m2 = oracle.Model.from_instance(small, phi_scale=2.0)
    r2, _, c2 = oracle.rates4(m2, [300.0], 1.0, 7, dq, targets)
    assert np.array_equal(c2, c7)
    assert np.array_equal(r2, 4.0 * r7)


def test_counts_monotone_in_scalebroad(small, small_model):
    """A smaller scalebroad admits fewer processes (Sec. 2.4): counts are non-decreasing in
    sb for every mode and channel."""
    dq = _dq(small)
    prev = None
    for sb in (0.05, 0.1, 0.3, 1.0, 2.0):
        _, _, c = oracle.rates4(small_model, [300.0], sb, 7, dq, want_rates=False)
        if prev is not None:
            assert np.all(c >= prev)
        prev = c
    assert prev.sum() > 0


def test_rates_high_temperature_scaling(small, small_model):
    """In the classical limit every occupation factor of Eq. 4phgamma grows as T^2, so
    rate(2T)/rate(T) -> 4 (catches a dropped /n0_lambda, which would give T^3)."""
    dq = _dq(small)
    targets = np.arange(3, small.nmodes, 29)
    r, _, _ = oracle.rates4(small_model, [1e6, 2e6], 1.0, 7, dq, targets)
    np.testing.assert_allclose(r[1] / r[0], 4.0, rtol=2e-3)


def test_inactive_modes_zero(small, small_model):
    """Gamma acoustic modes (omega = 0) get rate 0 and no processes."""
    r, _, c = oracle.rates4(small_model, [300.0], 1.0, 7, _dq(small), [0, 1, 2])
    assert np.all(r == 0) and np.all(c == 0)
