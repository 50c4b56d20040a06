"""Parity of the HIP three-phonon rate (Eq. 3phgamma, Eq. V3; a surrogate input feature)
with the FP64 CPU oracle, through the C ABI.

Bar: kept-process counts bit-exact (FP64 window predicate in a fixed order on both sides);
rates within 1e-10 relative (FP64 on both sides, only the summation order differs)."""
import itertools
import sys

import numpy as np
import pytest

import oracle
import synth
from synth.fc3 import FC3, random_fc3

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fp4():
    import paper_2104_04895_amd as m
    return m


def _ctx(fp4, inst, fc3):
    c = fp4.Context(0)
    c.load_lattice(inst.cr.A, inst.grid, inst.cr.mass, oracle.default_dq(inst.cr.A, inst.grid))
    c.load_modes(inst.omega, inst.evec, inst.vel)
    c.load_fc3(fc3.atoms, fc3.cells, fc3.phi)
    return c


def _oracle(inst, fc3, T, sb, targets=None):
    m = oracle.Model.from_instance(inst)
    return oracle.rates3(m, fc3, T, sb, oracle.default_dq(inst.cr.A, inst.grid), targets)


def _check(r, cnt, r_o, c_o):
    assert np.array_equal(cnt, c_o)
    scale = np.max(np.abs(r_o), axis=1, keepdims=True)
    err = np.abs(r - r_o) / np.maximum(np.abs(r_o), 1e-300)
    # entries far below the largest rate of their temperature are compared on that scale
    ok = (err <= RTOL) | (np.abs(r - r_o) <= RTOL * 1e-3 * scale)
    assert ok.all(), float(err.max())


def test_diamond_first_shell_all_modes(fp4):
    _say("case: rates3 diamond 3x3x3 26 triplets all modes, 2 T")
    inst = synth.diamond_instance((3, 3, 3), synth.configs.RC_FIRST, seed=21)
    fc3 = random_fc3(inst.cr, 3.0, np.random.default_rng(21))
    T = [300.0, 900.0]
    r_o, c_o = _oracle(inst, fc3, T, 1.0)
    with _ctx(fp4, inst, fc3) as c:
        r, cnt = c.compute_rates3(T, 1.0)
    assert c_o.sum() > 1000
    _check(r, cnt, r_o, c_o)


def test_diamond_second_shell_subset(fp4):
    _say("case: rates3 diamond 6x6x6 266 triplets subset, sb 0.5")
    inst = synth.diamond_instance((6, 6, 6), synth.configs.RC_FIRST, seed=23)
    fc3 = random_fc3(inst.cr, 4.0, np.random.default_rng(23))
    targets = np.arange(0, inst.nmodes, 11)
    r_o, c_o = _oracle(inst, fc3, [300.0], 0.5, targets)
    with _ctx(fp4, inst, fc3) as c:
        r, cnt = c.compute_rates3([300.0], 0.5, targets)
    _check(r, cnt, r_o, c_o)


@pytest.mark.parametrize("which", ["wurtzite", "layered"])
def test_four_atom_cells(fp4, which):
    _say(f"case: rates3 {which} 4-atom cell, small grid, subset")
    if which == "wurtzite":
        inst = synth.configs.wurtzite(grid=(3, 3, 2))
        fc3 = random_fc3(inst.cr, 3.4, np.random.default_rng(5))
    else:
        inst = synth.configs.layered(grid=(3, 3, 3))
        fc3 = random_fc3(inst.cr, 2.95, np.random.default_rng(6))
    targets = np.arange(1, inst.nmodes, 7)
    r_o, c_o = _oracle(inst, fc3, [300.0, 700.0], 1.0, targets)
    with _ctx(fp4, inst, fc3) as c:
        r, cnt = c.compute_rates3([300.0, 700.0], 1.0, targets)
    _check(r, cnt, r_o, c_o)


def test_one_atom_gamma_only(fp4):
    """N = 1, one atom: the closed-form case the oracle is pinned to (exact energy
    conservation, delta = 1 by the sigma floor)."""
    _say("case: rates3 one-atom gamma-only")
    import math
    rng = np.random.default_rng(10)
    C = rng.standard_normal((3, 3, 3))
    C = sum(np.transpose(C, p) for p in itertools.permutations(range(3))) / 6.0
    w = np.array([[10.0, 20.0, 30.0]])
    evec = np.zeros((1, 3, 1, 3), dtype=complex)
    for j in range(3):
        evec[0, j, 0, j] = 1.0
    fc3 = FC3(np.zeros((1, 3), np.int32), np.zeros((1, 2, 3), np.int32), C.reshape(1, 27))
    m = oracle.Model((1, 1, 1), [12.0], w, evec, np.zeros((1, 3, 3)), np.zeros((1, 4), np.int32),
                     np.zeros((1, 3, 3), np.int32), np.zeros((1, 81)))
    r_o, c_o = oracle.rates3(m, fc3, [400.0], 1.0, 0.3)
    with fp4.Context(0) as c:
        c.load_lattice(np.eye(3) * 3.0, (1, 1, 1), [12.0], 0.3)
        c.load_modes(w, evec, np.zeros((1, 3, 3)))
        c.load_fc3(fc3.atoms, fc3.cells, fc3.phi)
        r, cnt = c.compute_rates3([400.0], 1.0)
    assert np.array_equal(cnt, c_o)
    np.testing.assert_allclose(r, r_o, rtol=RTOL)


def test_training_grid_sampled(fp4):
    """12x12x12 grid (the surrogate's training size), first-shell FC3, 3 temperatures: all
    modes on the GPU, a sample against the oracle one mode at a time; gamma acoustic
    modes are zero."""
    _say("case: rates3 12x12x12 all modes, sampled oracle")
    inst = synth.diamond_instance((12, 12, 12), synth.configs.RC_FIRST, seed=24)
    fc3 = random_fc3(inst.cr, 3.0, np.random.default_rng(24))
    T = [100.0, 500.0, 1200.0]
    with _ctx(fp4, inst, fc3) as c:
        r, cnt = c.compute_rates3(T, 1.0)
    sample = np.random.default_rng(3).choice(inst.nmodes, size=24, replace=False)
    r_o, c_o = _oracle(inst, fc3, T, 1.0, sample)
    _check(r[:, sample], cnt[sample], r_o, c_o)
    assert np.all(r[:, :3] == 0) and np.all(cnt[:3] == 0)
    assert np.all(np.isfinite(r))


def test_rates3_argument_errors(fp4):
    _say("case: rates3 argument errors")
    inst = synth.diamond_instance((2, 2, 2), synth.configs.RC_FIRST, seed=25)
    with fp4.Context(0) as c:
        c.load_lattice(inst.cr.A, inst.grid, inst.cr.mass)
        c.load_modes(inst.omega, inst.evec, inst.vel)
        with pytest.raises(fp4.Fp4Error) as e:
            c.compute_rates3([300.0])
        assert e.value.code == fp4.FP4_E_STATE
        fc3 = random_fc3(inst.cr, 3.0, np.random.default_rng(1))
        bad = fc3.atoms.copy()
        bad[0, 1] = 2
        with pytest.raises(fp4.Fp4Error) as e:
            c.load_fc3(bad, fc3.cells, fc3.phi)
        assert e.value.code == fp4.FP4_E_INVAL
        c.load_fc3(fc3.atoms, fc3.cells, fc3.phi)
        with pytest.raises(fp4.Fp4Error):
            c.compute_rates3([300.0], 1.0, targets=[inst.nmodes])
        with pytest.raises(fp4.Fp4Error):
            c.compute_rates3([300.0], -1.0)
        r, cnt = c.compute_rates3([300.0], 1.0, targets=[5, 7])
        assert r.shape == (1, 2) and cnt.shape == (2, 2)


def test_three_atom_cell(fp4):
    _say("case: rates3 three-atom cell 3x3x2")
    from synth import configs
    inst = configs.three_atom(grid=(3, 3, 2))
    fc3 = random_fc3(inst.cr, 2.95, np.random.default_rng(8))
    targets = np.arange(2, inst.nmodes, 5)
    r_o, c_o = _oracle(inst, fc3, [300.0], 1.0, targets)
    with _ctx(fp4, inst, fc3) as c:
        r, cnt = c.compute_rates3([300.0], 1.0, targets)
    _check(r, cnt, r_o, c_o)
