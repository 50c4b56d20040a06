"""Brute-force four-phonon rates for tiny grids (test helper, independent of the oracle).

Differences from the oracle on purpose:
* q''' is not computed by folding: every grid point q''' is visited and an explicit
  Kronecker delta on q + s' q' + s'' q'' - q''' (mod the grid) selects the process;
* V of Eq. V4 is evaluated for all branch triples of a (q', q'', q''') block at once with a
  single einsum over quartets and Cartesian indices, with phases from numpy's exp.

The predicate uses the same left-to-right FP64 order (Python floats and numpy element-wise
ufuncs are IEEE double with no fused operations), so the kept-process sets must agree bit
for bit.
"""
from __future__ import annotations

import math

import numpy as np

from synth.crystal import grid_points

HBAR = 6.62607015e-34 / (2.0 * math.pi)
KB = 1.380649e-23
EV = 1.602176634e-19
AMU = 1.66053906660e-27

CHANNELS = [(+1, +1, 0.5), (+1, -1, 0.5), (-1, -1, 1.0 / 6.0)]


def c4_si() -> float:
    kv = EV / (1e-40 * AMU * AMU)
    return HBAR**2 * math.pi / 8.0 * kv * kv * 1e-72


def _phase(grid, n, R):
    f = (np.asarray(n)[None, :] * np.asarray(R)) / np.asarray(grid, dtype=float)
    return np.exp(2j * np.pi * f.sum(axis=-1))


def brute_rates(grid, mass, omega, evec, vel, atoms, cells, phi, T, sb, mask, dq, targets,
                W=2.0, sigma_min=1e-4):
    grid = tuple(int(g) for g in grid)
    pts = grid_points(grid)
    N = len(pts)
    nat = len(mass)
    nb = 3 * nat
    Phi = np.asarray(phi).reshape(-1, 3, 3, 3, 3)
    hk = HBAR / KB * 1e12
    C4 = c4_si()
    c_win = ((W * sb) * dq) * ((W * sb) * dq)
    c_sig = (sb * dq) * (sb * dq)
    om = omega.reshape(-1)
    ve = vel.reshape(-1, 3)
    T = np.atleast_1d(T)
    occ = np.zeros((len(T), om.size))
    for t, TT in enumerate(T):
        act = om > 0
        occ[t, act] = 1.0 / np.expm1(hk * om[act] / TT)
    sqm = np.sqrt(np.asarray(mass))
    ai, aj, ak, al = atoms.T
    Rj, Rk, Rl = cells[:, 0], cells[:, 1], cells[:, 2]

    def slot(iq, atom_idx, R, sign):
        # X[n, branch, x] = (e(q,branch)[atom_n][x] exp(i q.R_n))^(sign) / sqrt(M)
        ph = _phase(grid, pts[iq], R) if R is not None else np.ones(len(atom_idx))
        X = evec[iq][:, atom_idx, :] * ph[None, :, None] / sqm[atom_idx][None, :, None]
        X = np.transpose(X, (1, 0, 2))
        return X if sign > 0 else X.conj()

    rates = np.zeros((len(T), len(targets)))
    counts = np.zeros((len(targets), 3), dtype=np.int64)
    for it, mu in enumerate(targets):
        iq, j = divmod(int(mu), nb)
        if om[mu] <= 0.0:
            continue
        X1 = slot(iq, ai, None, +1)[:, j, :]
        for ch, (s1, s2, wch) in enumerate(CHANNELS):
            if not (mask >> ch) & 1:
                continue
            for iq1 in range(N):
                X2 = slot(iq1, aj, Rj, s1)
                for iq2 in range(N):
                    X3 = slot(iq2, ak, Rk, s2)
                    for iq3 in range(N):
                        dn = pts[iq] + s1 * pts[iq1] + s2 * pts[iq2] - pts[iq3]
                        if np.any(dn % np.asarray(grid) != 0):
                            continue          # explicit momentum Kronecker delta
                        X4 = slot(iq3, al, Rl, +1).conj()
                        V = np.einsum("nabcd,na,nxb,nyc,nzd->xyz", Phi, X1, X2, X3, X4,
                                      optimize=True)
                        for j1 in range(nb):
                            m1 = iq1 * nb + j1
                            if om[m1] <= 0:
                                continue
                            for j2 in range(nb):
                                m2 = iq2 * nb + j2
                                if om[m2] <= 0:
                                    continue
                                for j3 in range(nb):
                                    m3 = iq3 * nb + j3
                                    if om[m3] <= 0:
                                        continue
                                    a = om[mu] + om[m1] if s1 > 0 else om[mu] - om[m1]
                                    b = a + om[m2] if s2 > 0 else a - om[m2]
                                    dw = b - om[m3]
                                    dx = ve[m2, 0] - ve[m3, 0]
                                    dy = ve[m2, 1] - ve[m3, 1]
                                    dz = ve[m2, 2] - ve[m3, 2]
                                    s2v = (dx * dx + dy * dy) + dz * dz
                                    if not (dw * dw <= c_win * s2v):
                                        continue
                                    counts[it, ch] += 1
                                    sig2 = c_sig * s2v
                                    if sig2 < sigma_min * sigma_min:
                                        dlt = 1.0
                                    else:
                                        dlt = math.exp(-(dw * dw) / sig2) / (math.sqrt(math.pi) * math.sqrt(sig2))
                                    v2 = abs(V[j1, j2, j3]) ** 2
                                    wp = om[mu] * om[m1] * om[m2] * om[m3]
                                    for t in range(len(T)):
                                        n0 = occ[t]
                                        if ch == 0:
                                            f = (1 + n0[m1]) * (1 + n0[m2]) * n0[m3] / n0[mu]
                                        elif ch == 1:
                                            f = (1 + n0[m1]) * n0[m2] * n0[m3] / n0[mu]
                                        else:
                                            f = n0[m1] * n0[m2] * n0[m3] / n0[mu]
                                        rates[t, it] += wch * C4 / N**2 * f * v2 * dlt / wp
    return rates, counts


def c3_si() -> float:
    kv = EV / (1e-30 * AMU**1.5)
    return HBAR * math.pi / 4.0 * kv * kv * 1e-60


def brute_rates3(grid, mass, omega, evec, vel, atoms, cells, phi, T, sb, dq, targets,
                 W=2.0, sigma_min=1e-4):
    """Three-phonon rates (Eq. 3phgamma) by a double loop over q', q'' with an explicit
    momentum Kronecker delta on q +- q' - q''; V for all branch pairs by one einsum."""
    grid = tuple(int(g) for g in grid)
    pts = grid_points(grid)
    N = len(pts)
    nat = len(mass)
    nb = 3 * nat
    Phi = np.asarray(phi).reshape(-1, 3, 3, 3)
    hk = HBAR / KB * 1e12
    C3 = c3_si()
    c_win = ((W * sb) * dq) * ((W * sb) * dq)
    c_sig = (sb * dq) * (sb * dq)
    om = omega.reshape(-1)
    ve = vel.reshape(-1, 3)
    T = np.atleast_1d(T)
    occ = np.zeros((len(T), om.size))
    for t, TT in enumerate(T):
        act = om > 0
        occ[t, act] = 1.0 / np.expm1(hk * om[act] / TT)
    sqm = np.sqrt(np.asarray(mass))
    ai, aj, ak = atoms.T
    Rj, Rk = cells[:, 0], cells[:, 1]

    def slot(iq, atom_idx, R, sign):
        ph = _phase(grid, pts[iq], R) if R is not None else np.ones(len(atom_idx))
        X = evec[iq][:, atom_idx, :] * ph[None, :, None] / sqm[atom_idx][None, :, None]
        X = np.transpose(X, (1, 0, 2))
        return X if sign > 0 else X.conj()

    rates = np.zeros((len(T), len(targets)))
    counts = np.zeros((len(targets), 2), dtype=np.int64)
    for it, mu in enumerate(targets):
        iq, j = divmod(int(mu), nb)
        if om[mu] <= 0.0:
            continue
        X1 = slot(iq, ai, None, +1)[:, j, :]
        for ch, s1 in enumerate((+1, -1)):
            for iq1 in range(N):
                X2 = slot(iq1, aj, Rj, s1)
                for iq2 in range(N):
                    dn = pts[iq] + s1 * pts[iq1] - pts[iq2]
                    if np.any(dn % np.asarray(grid) != 0):
                        continue
                    X3 = slot(iq2, ak, Rk, +1).conj()
                    V = np.einsum("nabc,na,nxb,nyc->xy", Phi, X1, X2, X3, optimize=True)
                    for j1 in range(nb):
                        m1 = iq1 * nb + j1
                        if om[m1] <= 0:
                            continue
                        for j2 in range(nb):
                            m2 = iq2 * nb + j2
                            if om[m2] <= 0:
                                continue
                            a = om[mu] + om[m1] if s1 > 0 else om[mu] - om[m1]
                            dw = a - om[m2]
                            dx = ve[m1, 0] - ve[m2, 0]
                            dy = ve[m1, 1] - ve[m2, 1]
                            dz = ve[m1, 2] - ve[m2, 2]
                            s2v = (dx * dx + dy * dy) + dz * dz
                            if not (dw * dw <= c_win * s2v):
                                continue
                            counts[it, ch] += 1
                            sig2 = c_sig * s2v
                            if sig2 < sigma_min * sigma_min:
                                dlt = 1.0
                            else:
                                dlt = math.exp(-(dw * dw) / sig2) / (math.sqrt(math.pi) * math.sqrt(sig2))
                            v2 = abs(V[j1, j2]) ** 2
                            wp = om[mu] * om[m1] * om[m2]
                            for t in range(len(T)):
                                n0 = occ[t]
                                if ch == 0:
                                    rates[t, it] += C3 / N * (n0[m1] - n0[m2]) * v2 * dlt / wp
                                else:
                                    rates[t, it] += 0.5 * C3 / N * (n0[m1] + n0[m2] + 1) * v2 * dlt / wp
    return rates, counts
