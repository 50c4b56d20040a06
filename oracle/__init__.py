"""ctypes wrapper around the plain FP64 CPU oracle (oracle4.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the benchmark's
CPU-baseline leg.  The product library never imports, links or executes anything here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle4.c")
_LIB = os.path.join(_HERE, "liboracle4.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle4.c with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fcx-limited-range",
               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, u32, f64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
        L.oracle_rates4.argtypes = [P, i32, P, P, P, P, i32, P, P, P, P, i32, f64, u32, f64,
                                    f64, f64, i32, P, i32, P, P, P, i32]
        L.oracle_rates4.restype = ctypes.c_int
        L.oracle_phase_space4.argtypes = [P, i32, P, P, P, P, i32, P, P, P, P, i32, f64, u32,
                                          f64, f64, f64, i32, P, i32, P, P, P, i32]
        L.oracle_phase_space4.restype = ctypes.c_int
        L.oracle_rates4_class.argtypes = [P, i32, P, P, P, P, i32, P, P, P, P, i32, f64, u32,
                                          f64, f64, f64, i32, P, P, i32, i32, P, P, P, i32]
        L.oracle_rates4_class.restype = ctypes.c_int
        L.oracle_rates4_partners.argtypes = [P, i32, P, P, P, P, i32, P, P, P, P, i32, f64, u32,
                                             f64, f64, f64, i32, P, i32, P, i32, P, P, P, i32]
        L.oracle_rates4_partners.restype = ctypes.c_int
        L.oracle_rates3.argtypes = [P, i32, P, P, P, P, i32, P, P, P, P, i32, f64, f64, f64, f64,
                                    i32, P, P, P, i32]
        L.oracle_rates3.restype = ctypes.c_int
        L.oracle_v3.argtypes = [P, i32, P, P, P, P, i32, P, P, P, i32, P, P, P]
        L.oracle_v3.restype = ctypes.c_int
        L.oracle_c3.restype = f64
        L.oracle_c3.argtypes = []
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_kappa_rta.argtypes = [P, i32, P, P, P, P, i32, P, P, P, P]
        L.oracle_kappa_rta.restype = ctypes.c_int
        L.oracle_first_zone.argtypes = [P, P, i32, P, P]
        L.oracle_first_zone.restype = ctypes.c_int
        L.oracle_v4.argtypes = [P, i32, P, P, P, P, i32, P, P, P, i32, P, P, P]
        L.oracle_v4.restype = ctypes.c_int
        for name in ("oracle_hbar_over_kb", "oracle_c4"):
            getattr(L, name).restype = f64
            getattr(L, name).argtypes = []
        L.oracle_bose.restype = f64
        L.oracle_bose.argtypes = [f64, f64]
        L.oracle_delta.restype = f64
        L.oracle_delta.argtypes = [f64, f64, f64]
        L.oracle_default_dq.restype = f64
        L.oracle_default_dq.argtypes = [P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Model:
    """Contiguous copies of one instance's arrays in the layouts the oracle expects."""

    def __init__(self, grid, mass, omega, evec, vel, atoms, cells, phi):
        self.grid = np.ascontiguousarray(grid, dtype=np.int32)
        self.mass = np.ascontiguousarray(mass, dtype=np.float64)
        self.omega = np.ascontiguousarray(omega, dtype=np.float64)
        ev = np.ascontiguousarray(evec, dtype=np.complex128)
        self.evec = ev.view(np.float64)
        self.vel = np.ascontiguousarray(vel, dtype=np.float64)
        self.atoms = np.ascontiguousarray(atoms, dtype=np.int32)
        self.cells = np.ascontiguousarray(cells, dtype=np.int32)
        self.phi = np.ascontiguousarray(phi, dtype=np.float64)
        self.natoms = int(self.mass.shape[0])
        self.nb = 3 * self.natoms
        self.nq = int(np.prod(self.grid))

    @classmethod
    def from_instance(cls, inst, phi_scale: float = 1.0):
        return cls(inst.grid, inst.cr.mass, inst.omega, inst.evec, inst.vel, inst.fc4.atoms,
                   inst.fc4.cells, inst.fc4.phi * phi_scale)

    def _common(self):
        return [_p(self.grid), self.natoms, _p(self.mass), _p(self.omega), _p(self.evec),
                _p(self.vel), int(self.atoms.shape[0]), _p(self.atoms), _p(self.cells),
                _p(self.phi)]


def default_dq(A, grid) -> float:
    A = np.ascontiguousarray(A, dtype=np.float64)
    g = np.ascontiguousarray(grid, dtype=np.int32)
    return float(lib().oracle_default_dq(_p(A), _p(g)))


def rates4(model: Model, T, scalebroad, mask, dq, targets=None, window_w=2.0,
           sigma_min=1e-4, want_rates=True, nthreads=0):
    """Returns (rates[nT][nt], rates_ch[nT][3][nt], counts[nt][3])."""
    T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
    if targets is None:
        targets = np.arange(model.nq * model.nb)
    targets = np.ascontiguousarray(targets, dtype=np.int32)
    nt = int(targets.shape[0])
    rates = np.zeros((len(T), nt))
    rch = np.zeros((len(T), 3, nt))
    counts = np.zeros((nt, 3), dtype=np.int64)
    rc = lib().oracle_rates4(*model._common(), _p(T), len(T), float(scalebroad), int(mask),
                             float(window_w), float(sigma_min), float(dq), nt, _p(targets),
                             1 if want_rates else 0, _p(rates), _p(rch), _p(counts),
                             int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_rates4 returned {rc}")
    return rates, rch, counts


def phase_space4(model: Model, kind, T, scalebroad, mask, dq, targets=None, window_w=2.0,
                 sigma_min=1e-4, nthreads=0):
    """Four-phonon phase spaces (kind 1: weighted WP4, kind 2: P4), the rate sum with
    |V|^2 and the prefactor set to 1.  Returns (values[nT][nt], by_channel[nT][3][nt],
    counts[nt][3])."""
    T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
    if targets is None:
        targets = np.arange(model.nq * model.nb)
    targets = np.ascontiguousarray(targets, dtype=np.int32)
    nt = int(targets.shape[0])
    out = np.zeros((len(T), nt))
    och = np.zeros((len(T), 3, nt))
    counts = np.zeros((nt, 3), dtype=np.int64)
    rc = lib().oracle_phase_space4(*model._common(), _p(T), len(T), float(scalebroad), int(mask),
                                   float(window_w), float(sigma_min), float(dq), nt,
                                   _p(targets), int(kind), _p(out), _p(och), _p(counts),
                                   int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_phase_space4 returned {rc}")
    return out, och, counts


def rates4_class(model: Model, A, qclass, T, scalebroad, mask, dq, targets=None,
                 window_w=2.0, sigma_min=1e-4, want_rates=True, nthreads=0):
    """The rate sum restricted to normal (qclass 1, Q = 0) or Umklapp (qclass 2, Q != 0)
    processes, Q from the first-zone images of the four points (A: lattice vectors as rows).
    Returns (rates[nT][nt], rates_ch[nT][3][nt], counts[nt][3])."""
    T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
    if targets is None:
        targets = np.arange(model.nq * model.nb)
    targets = np.ascontiguousarray(targets, dtype=np.int32)
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
    nt = int(targets.shape[0])
    rates = np.zeros((len(T), nt))
    rch = np.zeros((len(T), 3, nt))
    counts = np.zeros((nt, 3), dtype=np.int64)
    rc = lib().oracle_rates4_class(*model._common(), _p(T), len(T), float(scalebroad), int(mask),
                                   float(window_w), float(sigma_min), float(dq), nt,
                                   _p(targets), _p(A), int(qclass), 1 if want_rates else 0,
                                   _p(rates), _p(rch), _p(counts), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_rates4_class returned {rc}")
    return rates, rch, counts


def rates4_partners(model: Model, T, scalebroad, mask, dq, targets, q1list, window_w=2.0,
                    sigma_min=1e-4, nthreads=0):
    """The rate sum restricted to partner points q' in q1list (a bounded sample of the work
    of the full sum).  Returns (rates[nT][nt], counts[nt][3])."""
    T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
    targets = np.ascontiguousarray(targets, dtype=np.int32)
    q1 = np.ascontiguousarray(q1list, dtype=np.int32)
    nt = int(targets.shape[0])
    rates = np.zeros((len(T), nt))
    rch = np.zeros((len(T), 3, nt))
    counts = np.zeros((nt, 3), dtype=np.int64)
    rc = lib().oracle_rates4_partners(*model._common(), _p(T), len(T), float(scalebroad),
                                      int(mask), float(window_w), float(sigma_min), float(dq),
                                      nt, _p(targets), len(q1), _p(q1), 1, _p(rates), _p(rch),
                                      _p(counts), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_rates4_partners returned {rc}")
    return rates, counts


def first_zone(A, grid, iq) -> np.ndarray:
    """First-zone images k[n][3] (Cartesian, 1/Angstrom) of the grid points iq, as the
    normal / Umklapp split uses them (A: lattice vectors as rows)."""
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
    g = np.ascontiguousarray(grid, dtype=np.int32)
    iq = np.ascontiguousarray(np.atleast_1d(iq), dtype=np.int32)
    k = np.zeros((len(iq), 3))
    rc = lib().oracle_first_zone(_p(A), _p(g), len(iq), _p(iq), _p(k))
    if rc != 0:
        raise ValueError(f"oracle_first_zone returned {rc}")
    return k


def v4(model: Model, modes4, signs4) -> np.ndarray:
    """V (Eq. V4) for explicit processes: modes4[n][4] mode ids, signs4[n][4] slot signs."""
    modes4 = np.ascontiguousarray(modes4, dtype=np.int32).reshape(-1, 4)
    signs4 = np.ascontiguousarray(signs4, dtype=np.int32).reshape(-1, 4)
    n = modes4.shape[0]
    V = np.zeros(n, dtype=np.complex128)
    lib().oracle_v4(*model._common(), n, _p(modes4), _p(signs4), _p(V.view(np.float64)))
    return V


def _fc3_args(model: Model, fc3):
    at = np.ascontiguousarray(fc3.atoms, dtype=np.int32)
    cl = np.ascontiguousarray(fc3.cells, dtype=np.int32)
    ph = np.ascontiguousarray(fc3.phi, dtype=np.float64)
    return [_p(model.grid), model.natoms, _p(model.mass), _p(model.omega), _p(model.evec),
            _p(model.vel), int(at.shape[0]), _p(at), _p(cl), _p(ph)], (at, cl, ph)


def rates3(model: Model, fc3, T, scalebroad, dq, targets=None, window_w=2.0, sigma_min=1e-4,
           nthreads=0):
    """Three-phonon rates (Eq. 3phgamma).  Returns (rates[nT][nt], counts[nt][2])."""
    T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
    if targets is None:
        targets = np.arange(model.nq * model.nb)
    targets = np.ascontiguousarray(targets, dtype=np.int32)
    nt = len(targets)
    rates = np.zeros((len(T), nt))
    counts = np.zeros((nt, 2), dtype=np.int64)
    args, keep = _fc3_args(model, fc3)
    rc = lib().oracle_rates3(*args, _p(T), len(T), float(scalebroad), float(window_w),
                             float(sigma_min), float(dq), nt, _p(targets), _p(rates), _p(counts),
                             int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_rates3 returned {rc}")
    return rates, counts


def v3(model: Model, fc3, modes3, signs3) -> np.ndarray:
    """V of Eq. V3 for explicit (mode, sign) triples."""
    modes3 = np.ascontiguousarray(modes3, dtype=np.int32).reshape(-1, 3)
    signs3 = np.ascontiguousarray(signs3, dtype=np.int32).reshape(-1, 3)
    V = np.zeros(len(modes3), dtype=np.complex128)
    args, keep = _fc3_args(model, fc3)
    lib().oracle_v3(*args, len(modes3), _p(modes3), _p(signs3), _p(V.view(np.float64)))
    return V


def max_threads() -> int:
    """OpenMP threads the oracle's parallel loops use by default."""
    return int(lib().oracle_max_threads())


def c3() -> float:
    return float(lib().oracle_c3())


def c4() -> float:
    return float(lib().oracle_c4())


def hbar_over_kb() -> float:
    return float(lib().oracle_hbar_over_kb())


def bose(omega, T) -> float:
    return float(lib().oracle_bose(float(omega), float(T)))


def delta(dw, sigma2, sigma_min=1e-4) -> float:
    return float(lib().oracle_delta(float(dw), float(sigma2), float(sigma_min)))


def kappa_rta(grid, natoms, omega, vel, A, T, rates3, rates4):
    """RTA thermal conductivity kappa[nT][3][3] (W/(m K)) from three- and four-phonon rates
    [nT][nmodes] (1/ps), and the number of active modes skipped for a zero total rate."""
    T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
    g = np.ascontiguousarray(grid, dtype=np.int32)
    om = np.ascontiguousarray(omega, dtype=np.float64).reshape(-1)
    v = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
    r3 = np.ascontiguousarray(rates3, dtype=np.float64).reshape(len(T), -1)
    r4 = np.ascontiguousarray(rates4, dtype=np.float64).reshape(len(T), -1)
    if r3.shape[1] != om.size or r4.shape[1] != om.size:
        raise ValueError("rates must be [nT][nmodes]")
    kappa = np.zeros((len(T), 3, 3))
    nskip = np.zeros(len(T), dtype=np.int64)
    rc = lib().oracle_kappa_rta(_p(g), int(natoms), _p(om), _p(v), _p(A), _p(T), len(T), _p(r3),
                                _p(r4), _p(kappa), _p(nskip))
    if rc != 0:
        raise ValueError(f"oracle_kappa_rta returned {rc}")
    return kappa, nskip
