"""Random fourth-order force constants with the symmetries the method relies on.

The rate formula needs a quartet list Phi_{ijkl}^{abgt} (atom i in the home cell) that is
* invariant under the 24 permutations of its (atom, Cartesian) slots, with the quartet
  re-anchored so that the first atom is again in the home cell (index-permutation symmetry);
* zero when summed over any one atom index (acoustic sum rule);
* covariant under the crystal's space group.

Instead of drawing independent numbers and projecting them onto those constraints, the
generator draws a random translation-invariant quartic energy for every cluster of atoms
whose pairwise distances are within the cutoff, and sums it over the space group and over
lattice translations.  The fourth derivative of such an energy has all three properties
by construction (permutation symmetry because it is a derivative of a scalar, the sum rule
because each cluster energy depends only on displacement differences, space-group
covariance because the energy is a group average).  The result is rescaled so that the
root-mean-square of the stored elements equals `rms` (eV/Angstrom^4).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from .crystal import Crystal, sites_within, distance, apply_op

_K = 6                 # cell components are encoded in [-_K, _K]
_NR = (2 * _K + 1) ** 3


@dataclass
class FC4:
    atoms: np.ndarray   # (n,4) int32 basis indices (i, j, k, l)
    cells: np.ndarray   # (n,3,3) int32 lattice coordinates of atoms j, k, l (atom i at 0)
    phi: np.ndarray     # (n,81) float64, index ((a*3+b)*3+g)*3+t, eV/Angstrom^4

    @property
    def n(self) -> int:
        return int(self.atoms.shape[0])


def _rcode(R):
    R = np.asarray(R)
    return (R[..., 0] + _K) + (2 * _K + 1) * ((R[..., 1] + _K) + (2 * _K + 1) * (R[..., 2] + _K))


def _qcode(ns, i, j, Rj, k, Rk, l, Rl):
    c = i
    c = c * ns + j
    c = c * _NR + _rcode(Rj)
    c = c * ns + k
    c = c * _NR + _rcode(Rk)
    c = c * ns + l
    c = c * _NR + _rcode(Rl)
    return c


def enumerate_quartets(cr: Crystal, rc: float):
    """All ordered quartets (i at home, j, k, l) whose six pairwise distances are <= rc
    (atoms may repeat).  Returns list of (i, (j,Rj), (k,Rk), (l,Rl))."""
    out = []
    for i in range(cr.natoms):
        home = (i, (0, 0, 0))
        nbrs = sites_within(cr, cr.position(*home), rc)
        for a, b, c in itertools.product(nbrs, repeat=3):
            if (distance(cr, a, b) <= rc + 1e-9 and distance(cr, a, c) <= rc + 1e-9
                    and distance(cr, b, c) <= rc + 1e-9):
                out.append((i, a, b, c))
    return out


def _canonical(cluster):
    best = None
    for (s0, R0) in cluster:
        shifted = sorted((s, tuple(np.subtract(R, R0))) for (s, R) in cluster)
        key = tuple(shifted)
        if best is None or key < best:
            best = key
    return best


def enumerate_clusters(cr: Crystal, rc: float, max_size: int = 4):
    """Sets of 2..max_size distinct sites, pairwise within rc, up to lattice translation."""
    seen = set()
    out = []
    for i in range(cr.natoms):
        home = (i, (0, 0, 0))
        nbrs = [x for x in sites_within(cr, cr.position(*home), rc) if x != home]
        for size in range(1, max_size):
            for sub in itertools.combinations(nbrs, size):
                ok = all(distance(cr, a, b) <= rc + 1e-9 for a, b in itertools.combinations(sub, 2))
                if not ok:
                    continue
                key = _canonical((home,) + sub)
                if key in seen:
                    continue
                seen.add(key)
                out.append(list(key))
    return out


def _sym4(C):
    out = np.zeros_like(C)
    for p in itertools.permutations(range(4)):
        out += np.transpose(C, p)
    return out / 24.0


def random_fc4(cr: Crystal, rc: float, rng: np.random.Generator, rms: float = 5.0) -> FC4:
    quartets = enumerate_quartets(cr, rc)
    ns = cr.natoms
    codes = np.array([_qcode(ns, i, j[0], j[1], k[0], k[1], l[0], l[1])
                      for (i, j, k, l) in quartets], dtype=np.int64)
    order = np.argsort(codes)
    codes = codes[order]
    quartets = [quartets[o] for o in order]
    index = {int(c): n for n, c in enumerate(codes)}
    phi = np.zeros((len(quartets), 3, 3, 3, 3))

    for cluster in enumerate_clusters(cr, rc):
        m = len(cluster)
        d = 3 * (m - 1)
        C = _sym4(rng.standard_normal((d, d, d, d)))
        # displacement differences: Delta_k = u_k - u_0 (k = 1..m-1)
        Dm = np.zeros((m - 1, 3, m, 3))
        for kk in range(1, m):
            for x in range(3):
                Dm[kk - 1, x, kk, x] = 1.0
                Dm[kk - 1, x, 0, x] = -1.0
        Dm = Dm.reshape(d, m, 3)
        # Phi_c[a,al,b,be,c,ga,d,th] in (site, cartesian) slots
        P = np.einsum("KLMN,Kai,Lbj,Mck,Ndl->aibjckdl", C, Dm, Dm, Dm, Dm, optimize=True)
        tuples = np.array(list(itertools.product(range(m), repeat=4)))
        for op in cr.ops:
            T = op[0]
            img = [apply_op(cr, op, site) for site in cluster]
            s_img = np.array([x[0] for x in img])
            R_img = np.array([x[1] for x in img])
            Pr = np.einsum("ai,bj,ck,dl,xiyjzkwl->xaybzcwd", T, T, T, T, P, optimize=True)
            ta, tb, tc, td = tuples.T
            R0 = R_img[ta]
            qc = _qcode(ns, s_img[ta], s_img[tb], R_img[tb] - R0, s_img[tc], R_img[tc] - R0,
                        s_img[td], R_img[td] - R0)
            idx = np.array([index[int(c)] for c in qc])
            vals = Pr[ta, :, tb, :, tc, :, td, :]
            np.add.at(phi, idx, vals)

    phi = phi.reshape(len(quartets), 81)
    scale = rms / np.sqrt(np.mean(phi**2))
    phi *= scale
    atoms = np.array([[i, j[0], k[0], l[0]] for (i, j, k, l) in quartets], dtype=np.int32)
    cells = np.array([[j[1], k[1], l[1]] for (i, j, k, l) in quartets], dtype=np.int32)
    return FC4(atoms, cells, phi)


def scaled(fc: FC4, factor: float) -> FC4:
    return FC4(fc.atoms.copy(), fc.cells.copy(), fc.phi * factor)


def single_component(atoms, cells, comp, value) -> FC4:
    """A one-quartet, one-component FC4 (used for closed-form checks)."""
    phi = np.zeros((1, 81))
    phi[0, comp] = value
    return FC4(np.asarray([atoms], dtype=np.int32), np.asarray([cells], dtype=np.int32), phi)
