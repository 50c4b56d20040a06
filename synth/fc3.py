"""Random third-order force constants (input of the three-phonon rate feature).

Same construction as the fourth-order list: a random translation-invariant cubic energy on
every cluster of <= 3 atoms with pairwise distances within the cutoff, summed over the space
group and lattice translations, so that the triplet list is permutation symmetric, satisfies
the acoustic sum rule and is space-group covariant.  Rescaled to a given RMS (eV/A^3).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from .crystal import Crystal, sites_within, distance, apply_op
from .fc4 import _rcode, _NR, enumerate_clusters


@dataclass
class FC3:
    atoms: np.ndarray   # (n,3) int32 basis indices (i, j, k)
    cells: np.ndarray   # (n,2,3) int32 lattice coordinates of atoms j, k (atom i at 0)
    phi: np.ndarray     # (n,27) float64, index (a*3+b)*3+g, eV/Angstrom^3

    @property
    def n(self) -> int:
        return int(self.atoms.shape[0])


def _tcode(ns, i, j, Rj, k, Rk):
    c = i
    c = c * ns + j
    c = c * _NR + _rcode(Rj)
    c = c * ns + k
    c = c * _NR + _rcode(Rk)
    return c


def enumerate_triplets(cr: Crystal, rc: float):
    out = []
    for i in range(cr.natoms):
        home = (i, (0, 0, 0))
        nbrs = sites_within(cr, cr.position(*home), rc)
        for a, b in itertools.product(nbrs, repeat=2):
            if distance(cr, a, b) <= rc + 1e-9:
                out.append((i, a, b))
    return out


def _sym3(C):
    out = np.zeros_like(C)
    for p in itertools.permutations(range(3)):
        out += np.transpose(C, p)
    return out / 6.0


def random_fc3(cr: Crystal, rc: float, rng: np.random.Generator, rms: float = 10.0) -> FC3:
    trip = enumerate_triplets(cr, rc)
    ns = cr.natoms
    codes = np.array([_tcode(ns, i, j[0], j[1], k[0], k[1]) for (i, j, k) in trip], dtype=np.int64)
    order = np.argsort(codes)
    codes = codes[order]
    trip = [trip[o] for o in order]
    index = {int(c): n for n, c in enumerate(codes)}
    phi = np.zeros((len(trip), 3, 3, 3))
    for cluster in enumerate_clusters(cr, rc, max_size=3):
        m = len(cluster)
        d = 3 * (m - 1)
        C = _sym3(rng.standard_normal((d, d, d)))
        Dm = np.zeros((m - 1, 3, m, 3))
        for kk in range(1, m):
            for x in range(3):
                Dm[kk - 1, x, kk, x] = 1.0
                Dm[kk - 1, x, 0, x] = -1.0
        Dm = Dm.reshape(d, m, 3)
        P = np.einsum("KLM,Kai,Lbj,Mck->aibjck", C, Dm, Dm, Dm, optimize=True)
        tuples = np.array(list(itertools.product(range(m), repeat=3)))
        for op in cr.ops:
            T = op[0]
            img = [apply_op(cr, op, site) for site in cluster]
            s_img = np.array([x[0] for x in img])
            R_img = np.array([x[1] for x in img])
            Pr = np.einsum("ai,bj,ck,xiyjzk->xaybzc", T, T, T, P, optimize=True)
            ta, tb, tc = tuples.T
            R0 = R_img[ta]
            qc = _tcode(ns, s_img[ta], s_img[tb], R_img[tb] - R0, s_img[tc], R_img[tc] - R0)
            idx = np.array([index[int(c)] for c in qc])
            np.add.at(phi, idx, Pr[ta, :, tb, :, tc, :])
    phi = phi.reshape(len(trip), 27)
    phi *= rms / np.sqrt(np.mean(phi**2))
    atoms = np.array([[i, j[0], k[0]] for (i, j, k) in trip], dtype=np.int32)
    cells = np.array([[j[1], k[1]] for (i, j, k) in trip], dtype=np.int32)
    return FC3(atoms, cells, phi)
