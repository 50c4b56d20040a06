"""Seeded synthetic workloads.

Every workload is built from a structure, a Born-von Karman spring model, a Gamma-centred
grid and a random symmetric FC4 list (see `fc4.py`).  The seeds below fix every draw.

* ``small``  : diamond-structure 2-atom cell (mass 28, a = 5.43 A), 3x3x3 grid,
               first-shell FC4 (r_c = 3.0 A, 58 quartets), T = 300 K, scalebroad 1.
* ``medium`` : same model, 8x8x8 grid, FC4 out to the second shell (r_c = 4.2 A),
               T = 300 and 1000 K.
* ``large``  : same model, 16x16x16 grid, second-shell FC4, T = 300 K.
* ``wurtzite`` / ``layered`` / ``cubic10`` : the uneven instances of the batched workload.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import crystal as cx
from .harmonic import bvk_fc2, modes
from .fc4 import FC4, random_fc4


@dataclass
class Instance:
    name: str
    cr: cx.Crystal
    grid: tuple
    omega: np.ndarray     # (nq, nb) rad/ps
    evec: np.ndarray      # (nq, nb, nat, 3) complex128
    vel: np.ndarray       # (nq, nb, 3) A/ps
    fc4: FC4
    T: list = field(default_factory=lambda: [300.0])
    scalebroad: float = 1.0
    mask: int = 7

    @property
    def nq(self) -> int:
        return int(np.prod(self.grid))

    @property
    def nb(self) -> int:
        return self.cr.nb

    @property
    def nmodes(self) -> int:
        return self.nq * self.nb


DIAMOND_SPRINGS = [(2.6, 10.0), (4.0, 1.0)]   # (max distance in A, k in eV/A^2) per shell
RC_FIRST = 3.0
RC_SECOND = 4.2

_FC4_CACHE: dict = {}


def _fc4_cached(cr, rc, seed):
    key = (cr.name, rc, seed)
    if key not in _FC4_CACHE:
        _FC4_CACHE[key] = random_fc4(cr, rc, np.random.default_rng(seed))
    return _FC4_CACHE[key]


def diamond_instance(grid, rc, seed, T=(300.0,), scalebroad=1.0, mask=7, name=None,
                     fc4_seed=None) -> Instance:
    cr = cx.diamond()
    rng = np.random.default_rng(seed)
    fc2 = bvk_fc2(cr, DIAMOND_SPRINGS, rng)
    om, ev, ve = modes(cr, fc2, tuple(grid))
    fc = _fc4_cached(cr, rc, seed if fc4_seed is None else fc4_seed)
    return Instance(name or f"diamond{grid[0]}x{grid[1]}x{grid[2]}", cr, tuple(grid), om, ev,
                    ve, fc, list(T), scalebroad, mask)


def small(seed: int = 1) -> Instance:
    return diamond_instance((3, 3, 3), RC_FIRST, seed, (300.0,), 1.0, 7, "small-3x3x3")


def medium(seed: int = 2) -> Instance:
    return diamond_instance((8, 8, 8), RC_SECOND, seed, (300.0, 1000.0), 1.0, 7, "medium-8x8x8")


def large(seed: int = 3) -> Instance:
    return diamond_instance((16, 16, 16), RC_SECOND, seed, (300.0,), 1.0, 7, "large-16x16x16")


def wurtzite(seed: int = 42, grid=(8, 8, 6)) -> Instance:
    cr = cx.wurtzite_like()
    rng = np.random.default_rng(seed)
    fc2 = bvk_fc2(cr, [(2.2, 10.0), (3.4, 1.0)], rng)
    om, ev, ve = modes(cr, fc2, tuple(grid))
    fc = random_fc4(cr, 3.4, np.random.default_rng(seed + 1000))
    return Instance("wurtzite-8x8x6", cr, tuple(grid), om, ev, ve, fc, [300.0, 700.0])


def layered(seed: int = 43, grid=(6, 6, 6)) -> Instance:
    cr = cx.layered_rhombohedral()
    rng = np.random.default_rng(seed)
    fc2 = bvk_fc2(cr, [(2.3, 10.0), (3.0, 1.0)], rng)
    om, ev, ve = modes(cr, fc2, tuple(grid))
    fc = random_fc4(cr, 2.95, np.random.default_rng(seed + 1000))
    return Instance("layered-6x6x6", cr, tuple(grid), om, ev, ve, fc, [300.0, 700.0])


def three_atom(seed: int = 44, grid=(3, 3, 3)) -> Instance:
    cr = cx.layered_three_atom()
    rng = np.random.default_rng(seed)
    fc2 = bvk_fc2(cr, [(2.3, 10.0), (3.0, 1.0)], rng)
    om, ev, ve = modes(cr, fc2, tuple(grid))
    fc = random_fc4(cr, 2.95, np.random.default_rng(seed + 1000))
    return Instance(f"three-atom-{grid[0]}x{grid[1]}x{grid[2]}", cr, tuple(grid), om, ev, ve, fc,
                    [300.0, 700.0])


def one_atom(seed: int = 45, grid=(4, 4, 4)) -> Instance:
    cr = cx.fcc_one_atom()
    rng = np.random.default_rng(seed)
    fc2 = bvk_fc2(cr, [(2.55, 10.0), (3.6, 1.0)], rng)
    om, ev, ve = modes(cr, fc2, tuple(grid))
    fc = random_fc4(cr, 2.6, np.random.default_rng(seed + 1000))
    return Instance(f"fcc-one-atom-{grid[0]}x{grid[1]}x{grid[2]}", cr, tuple(grid), om, ev, ve,
                    fc, [300.0, 700.0])


def ortho(seed: int = 46, grid=(4, 3, 2)) -> Instance:
    cr = cx.ortho_one_atom()
    rng = np.random.default_rng(seed)
    fc2 = bvk_fc2(cr, [(3.0, 10.0), (3.3, 8.0), (3.6, 6.0)], rng)
    om, ev, ve = modes(cr, fc2, tuple(grid))
    fc = random_fc4(cr, 3.65, np.random.default_rng(seed + 1000))
    return Instance(f"ortho-one-atom-{grid[0]}x{grid[1]}x{grid[2]}", cr, tuple(grid), om, ev, ve,
                    fc, [300.0, 700.0])


def cubic10(seed: int = 41) -> Instance:
    inst = diamond_instance((10, 10, 10), RC_SECOND, seed, (300.0, 700.0), 1.0, 7, "cubic-10x10x10")
    return inst
