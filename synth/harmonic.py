"""Born-von Karman harmonic model and phonon modes on a Gamma-centred grid.

Builds the inputs of the rate calculation: frequencies omega[nq][nb] (rad/ps), eigenvectors
e[nq][nb][nat][3] (complex, unit norm) and group velocities v[nq][nb][3] (Angstrom/ps).

Conventions (these fix what the matrix-element formula assumes of its inputs):
* D(q)_{a alpha, b beta} = sum_R Phi2(0a, Rb)_{alpha beta} exp(+i q.R) / sqrt(M_a M_b), with
  R the lattice vector of the cell holding atom b (phases on lattice vectors only).
* e(-q) = conj(e(q)) exactly (time-reversal gauge); at q equivalent to -q the dynamical
  matrix is real and the eigenvectors are taken real.
* The three acoustic modes at Gamma have omega = 0.0 exactly and the eigenvectors of rigid
  translations.
* Velocities are Hellmann-Feynman derivatives averaged over degenerate sets; v(-q) = -v(q)
  exactly and v = 0 at q equivalent to -q.
"""
from __future__ import annotations

import numpy as np

from .crystal import Crystal, sites_within, grid_points, minus_index, bloch_phase
from .units import OMEGA_UNIT


def bvk_fc2(cr: Crystal, shells, rng: np.random.Generator, bend_ratio: float = 0.25,
            spread: float = 0.10):
    """Bond springs: for every pair at distance d <= rmax of a shell (rmax, k), the 3x3
    block Phi2(a, b) = -(k_s rr^T + b_s (I - rr^T)) with k_s = k (1 + spread u) and
    b_s = bend_ratio * k (1 + spread u'), u, u' ~ U(-1, 1) drawn ONCE per shell, so the
    model keeps every symmetry of the structure.  Self blocks enforce the sum rule.
    Returns dict {(a, b, R): 3x3}."""
    params = []
    for (rmax, k) in shells:
        u, up = rng.uniform(-1.0, 1.0, size=2)
        params.append((rmax, k * (1.0 + spread * u), bend_ratio * k * (1.0 + spread * up)))
    fc = {}
    rmax_all = max(r for r, _ in shells)
    for a in range(cr.natoms):
        ra = cr.position(a, (0, 0, 0))
        self_blk = np.zeros((3, 3))
        for (b, R) in sites_within(cr, ra, rmax_all):
            d = cr.position(b, R) - ra
            dist = np.linalg.norm(d)
            if dist < 1e-8:
                continue
            for (rmax, ks, bs) in params:
                if dist <= rmax + 1e-9:
                    rr = np.outer(d, d) / dist**2
                    blk = -(ks * rr + bs * (np.eye(3) - rr))
                    fc[(a, b, R)] = fc.get((a, b, R), np.zeros((3, 3))) + blk
                    self_blk -= blk
                    break
        fc[(a, a, (0, 0, 0))] = fc.get((a, a, (0, 0, 0)), np.zeros((3, 3))) + self_blk
    return fc


def dynmat(cr: Crystal, fc2, grid, n):
    """D(q) and dD/dq (Cartesian, 3 matrices) at integer grid point n."""
    nat = cr.natoms
    D = np.zeros((3 * nat, 3 * nat), dtype=complex)
    dD = np.zeros((3, 3 * nat, 3 * nat), dtype=complex)
    n = np.asarray(n)
    for (a, b, R), blk in fc2.items():
        Rv = np.asarray(R)
        ph = bloch_phase(grid, n[None, :], Rv[None, :])[0]
        w = blk / np.sqrt(cr.mass[a] * cr.mass[b])
        D[3 * a:3 * a + 3, 3 * b:3 * b + 3] += w * ph
        Rc = Rv @ cr.A
        for x in range(3):
            dD[x, 3 * a:3 * a + 3, 3 * b:3 * b + 3] += 1j * Rc[x] * w * ph
    return D, dD


def _degenerate_sets(w, tol):
    sets, cur = [], [0]
    for j in range(1, len(w)):
        if abs(w[j] - w[cur[-1]]) <= tol:
            cur.append(j)
        else:
            sets.append(cur)
            cur = [j]
    sets.append(cur)
    return sets


def rotate_index(cr: Crystal, grid, T, iq):
    """Grid index of T q (Cartesian rotation T), or None if T q is not on the grid."""
    g = np.asarray(grid, dtype=float)
    n = grid_points(grid)[iq] / g
    f = (T @ (n @ cr.B)) @ cr.A.T / (2.0 * np.pi) * g
    fi = np.rint(f)
    if np.max(np.abs(f - fi)) > 1e-8:
        return None
    fi = fi.astype(np.int64) % np.asarray(grid)
    return int(fi[0] + grid[0] * (fi[1] + grid[1] * fi[2]))


def _solve(cr, fc2, grid, n, selfpair, transl, iq_is_gamma):
    D, dD = dynmat(cr, fc2, grid, n)
    D = 0.5 * (D + D.conj().T)
    if selfpair:
        lam, U = np.linalg.eigh(D.real)
        U = U.astype(complex)
    else:
        lam, U = np.linalg.eigh(D)
    if np.min(lam) < -1e-8 * max(1.0, np.max(np.abs(lam))):
        raise ValueError(f"unstable harmonic model at q = {n}: {lam.min()}")
    w = OMEGA_UNIT * np.sqrt(np.clip(lam, 0.0, None))
    if iq_is_gamma:
        # acoustic modes at Gamma: exact zeros and rigid translations; optical block
        # re-diagonalised in the complement of the translations
        w[:3] = 0.0
        Q = U[:, 3:] - transl.T @ (transl @ U[:, 3:])
        Q, _ = np.linalg.qr(Q)
        Dp = Q.conj().T @ D @ Q
        Dp = 0.5 * (Dp + Dp.conj().T)
        l2, V2 = np.linalg.eigh(Dp.real)
        U = np.concatenate([transl.T.astype(complex), Q @ V2], axis=1)
        w[3:] = OMEGA_UNIT * np.sqrt(np.clip(l2, 0.0, None))
        if selfpair:
            U = U.real.astype(complex)
    return w, U, dD


def modes(cr: Crystal, fc2, grid, degen_tol: float = 1e-6):
    """omega[nq][nb], evec[nq][nb][nat][3] complex, vel[nq][nb][3] on the full grid.

    Frequencies inside a degenerate set are made bitwise equal (their mean) and the
    frequencies and velocities of every q in a star are copied from its representative
    (velocities rotated by the operation, which for signed-permutation rotations is exact),
    so that every energy-window decision is exactly symmetric.  Eigenvectors are computed
    at every q."""
    nat, nb = cr.natoms, cr.nb
    grid = tuple(int(x) for x in grid)
    pts = grid_points(grid)
    nq = len(pts)
    mq = minus_index(grid)
    omega = np.zeros((nq, nb))
    evec = np.zeros((nq, nb, nat, 3), dtype=complex)
    vel = np.zeros((nq, nb, 3))
    done = np.zeros(nq, dtype=bool)
    transl = np.zeros((3, nb))
    msum = cr.mass.sum()
    for x in range(3):
        for a in range(nat):
            transl[x, 3 * a + x] = np.sqrt(cr.mass[a] / msum)
    rots = [op[0] for op in cr.ops] or [np.eye(3)]
    for rep in range(nq):
        if done[rep]:
            continue
        selfpair = mq[rep] == rep
        w, U, dD = _solve(cr, fc2, grid, pts[rep], selfpair, transl, rep == 0)
        tol = degen_tol * max(1.0, w.max())
        sets = _degenerate_sets(w, tol)
        for s in sets:
            if len(s) > 1:
                w[s] = np.mean(w[s])
        v = np.zeros((nb, 3))
        if not selfpair:
            for j in range(nb):
                if w[j] > 0.0:
                    for x in range(3):
                        v[j, x] = (OMEGA_UNIT**2) * np.real(U[:, j].conj() @ dD[x] @ U[:, j]) / (2.0 * w[j])
            for s in sets:
                v[s] = v[s].mean(axis=0)
        # star of rep: every rotation image and its time-reversed partner
        for T in rots:
            img = rotate_index(cr, grid, T, rep)
            if img is None or done[img]:
                continue
            if img == rep:
                Ui = U
            else:
                _, Ui, _ = _solve(cr, fc2, grid, pts[img], mq[img] == img, transl, False)
            vi = v @ T.T
            omega[img], evec[img], vel[img] = w, Ui.T.reshape(nb, nat, 3), vi
            done[img] = True
            m = mq[img]
            if not done[m]:
                omega[m] = w
                evec[m] = Ui.T.reshape(nb, nat, 3).conj()
                vel[m] = -vi
                done[m] = True
    return omega, evec, vel
