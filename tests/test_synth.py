"""Checks of the seeded input generator: the harmonic modes and FC4 have the properties the
rate formula assumes of its inputs."""
from collections import defaultdict

import numpy as np
import pytest

import synth
from synth.crystal import apply_op, grid_points, minus_index, sites_within
from synth.fc4 import _qcode
from synth.harmonic import bvk_fc2, dynmat
from synth.units import OMEGA_UNIT


@pytest.fixture(scope="module")
def inst():
    return synth.diamond_instance((4, 4, 4), synth.configs.RC_SECOND, seed=21)


def test_counts_of_quartets():
    cr = synth.diamond()
    assert synth.random_fc4(cr, 3.0, np.random.default_rng(0)).n == 58
    assert synth.random_fc4(cr, 4.2, np.random.default_rng(0)).n == 1522


def test_modes_orthonormal_and_time_reversal(inst):
    ev = inst.evec.reshape(inst.nq, inst.nb, inst.nb)
    for iq in range(inst.nq):
        G = ev[iq].conj() @ ev[iq].T
        assert np.max(np.abs(G - np.eye(inst.nb))) < 1e-12
    mq = minus_index(inst.grid)
    assert np.array_equal(inst.evec[mq], inst.evec.conj())
    assert np.array_equal(inst.omega[mq], inst.omega)
    assert np.array_equal(inst.vel[mq], -inst.vel)
    assert np.all(inst.omega[0, :3] == 0.0)
    assert np.all(inst.omega[1:] > 0.0)


def test_eigen_equation(inst):
    rng = np.random.default_rng(0)
    fc2 = bvk_fc2(inst.cr, synth.configs.DIAMOND_SPRINGS, np.random.default_rng(21))
    pts = grid_points(inst.grid)
    for iq in rng.choice(inst.nq, 6, replace=False):
        D, _ = dynmat(inst.cr, fc2, inst.grid, pts[iq])
        assert np.max(np.abs(D - D.conj().T)) < 1e-12
        U = inst.evec[iq].reshape(inst.nb, inst.nb).T
        lam = (inst.omega[iq] / OMEGA_UNIT) ** 2
        assert np.max(np.abs(D @ U - U * lam[None, :])) < 1e-8


def test_bloch_consistency(inst):
    """e_b(q) exp(i q.R) / sqrt(M_b) is an eigenvector of the real-space supercell force
    matrix: this pins the sign of the phase in D(q) that Eq. V4 assumes (with exp(-i q.R)
    the residual is O(1))."""
    cr = inst.cr
    fc2 = bvk_fc2(cr, synth.configs.DIAMOND_SPRINGS, np.random.default_rng(21))
    grid = np.asarray(inst.grid)
    cells = grid_points(inst.grid)
    nc, nat = len(cells), cr.natoms
    big = np.zeros((nc * nat * 3, nc * nat * 3))
    cidx = {tuple(c): k for k, c in enumerate(cells)}
    for k, c in enumerate(cells):
        for (a, b, R), blk in fc2.items():
            c2 = tuple((c + np.asarray(R)) % grid)
            i0 = (k * nat + a) * 3
            j0 = (cidx[c2] * nat + b) * 3
            big[i0:i0 + 3, j0:j0 + 3] += blk
    pts = grid_points(inst.grid)
    for iq in (5, 17, 42):
        q = pts[iq] / grid
        for j in (1, 4):
            u = np.zeros(nc * nat * 3, dtype=complex)
            for k, c in enumerate(cells):
                ph = np.exp(2j * np.pi * np.dot(q, c))
                for a in range(nat):
                    u[(k * nat + a) * 3:(k * nat + a) * 3 + 3] = inst.evec[iq, j, a] * ph / np.sqrt(cr.mass[a])
            lhs = big @ u
            Mu = np.repeat(np.tile(cr.mass, nc), 3) * u
            lam = (inst.omega[iq, j] / OMEGA_UNIT) ** 2
            assert np.max(np.abs(lhs - lam * Mu)) < 1e-9 * np.max(np.abs(lhs))


def test_velocities_finite_difference():
    """Hellmann-Feynman velocities against a central difference of omega on a fine grid
    (non-degenerate bands only)."""
    cr = synth.diamond()
    fc2 = bvk_fc2(cr, synth.configs.DIAMOND_SPRINGS, np.random.default_rng(3))
    grid = (4000, 4000, 4000)
    n0 = np.array([460, 1220, 140])
    from synth.harmonic import _solve
    transl = np.zeros((3, 6))
    w0, U, dD = _solve(cr, fc2, grid, n0, False, transl, False)
    for x in range(3):
        e = np.zeros(3, dtype=int)
        e[x] = 1
        wp, _, _ = _solve(cr, fc2, grid, n0 + e, False, transl, False)
        wm, _, _ = _solve(cr, fc2, grid, n0 - e, False, transl, False)
        dq = cr.B[x] / grid[x]
        for j in range(6):
            if min(abs(w0[j] - w0[k]) for k in range(6) if k != j) < 1.0:
                continue
            v = OMEGA_UNIT**2 * np.real(U[:, j].conj() @ dD @ U[:, j]) / (2 * w0[j])
            fd = (wp[j] - wm[j]) / 2.0
            assert np.dot(v, dq) == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_fc4_permutation_asr_and_space_group(inst):
    cr, fc = inst.cr, inst.fc4
    A = fc.atoms.astype(np.int64)
    C = fc.cells.astype(np.int64)
    ns = 2
    idx = {int(_qcode(ns, A[n, 0], A[n, 1], C[n, 0], A[n, 2], C[n, 1], A[n, 3], C[n, 2])): n for n in range(fc.n)}
    P = fc.phi.reshape(-1, 3, 3, 3, 3)
    scale = np.abs(P).max()
    # permutation symmetry with re-anchoring
    import itertools
    for n in range(0, fc.n, 7):
        sites = [(A[n, 0], np.zeros(3, dtype=np.int64))] + [(A[n, s], C[n, s - 1]) for s in (1, 2, 3)]
        for p in itertools.permutations(range(4)):
            ps = [sites[k] for k in p]
            R0 = ps[0][1]
            code = int(_qcode(ns, ps[0][0], ps[1][0], ps[1][1] - R0, ps[2][0], ps[2][1] - R0,
                              ps[3][0], ps[3][1] - R0))
            assert np.max(np.abs(np.transpose(P[n], p) - P[idx[code]])) < 1e-12 * scale
    # acoustic sum rule over the last atom (all atoms and cells)
    acc = defaultdict(lambda: np.zeros((3, 3, 3, 3)))
    for n in range(fc.n):
        acc[(A[n, 0], A[n, 1], tuple(C[n, 0]), A[n, 2], tuple(C[n, 1]))] += P[n]
    assert max(np.abs(v).max() for v in acc.values()) < 1e-12 * scale * 10
    # space-group covariance (Eq. SGSO)
    for op in cr.ops[::5]:
        T = op[0]
        for n in range(0, fc.n, 11):
            sites = [(int(A[n, 0]), (0, 0, 0))] + [(int(A[n, s]), tuple(int(x) for x in C[n, s - 1])) for s in (1, 2, 3)]
            img = [apply_op(cr, op, s) for s in sites]
            R0 = np.array(img[0][1])
            code = int(_qcode(ns, img[0][0], img[1][0], np.array(img[1][1]) - R0, img[2][0],
                              np.array(img[2][1]) - R0, img[3][0], np.array(img[3][1]) - R0))
            rot = np.einsum("ai,bj,ck,dl,ijkl->abcd", T, T, T, T, P[n])
            assert np.max(np.abs(rot - P[idx[code]])) < 1e-12 * scale


def test_fc4_rms():
    fc = synth.random_fc4(synth.diamond(), 3.0, np.random.default_rng(1))
    assert np.sqrt(np.mean(fc.phi**2)) == pytest.approx(5.0, rel=1e-12)


def test_other_structures_build():
    for maker in (synth.configs.wurtzite, synth.configs.layered):
        inst = maker(grid=(2, 2, 2))
        assert inst.nb == 12
        assert np.all(inst.omega[1:] > 0)
        assert inst.fc4.n > 0
