"""Pins of the oracle's RTA thermal conductivity (three- plus four-phonon relaxation time,
Eq. tao0 without the isotope term; F = tau v, Eq. BTE in the relaxation-time approximation).

* SI closed form: one q point, three modes of equal frequency moving along x, y and z with
  speed v and rate r: kappa = k_B E(x) v^2 / (r Omega) I with the Einstein heat-capacity
  function E(x) = x^2 e^x / (e^x - 1)^2 (1 in the classical limit), here written with numpy's
  exp and units converted by hand (A/ps = 100 m/s, ps = 1e-12 s, A^3 = 1e-30 m^3).
* Matthiessen's rule: only the total rate matters (any split between 3ph and 4ph gives the
  same kappa), and doubling it halves kappa exactly.
* Cubic isotropy: on the diamond-structure 3x3x3 workload with the oracle's own 3ph and 4ph
  rates, kappa is a multiple of the identity (off-diagonal and anisotropic parts at the
  rounding level).
* Modes with zero total rate are left out and counted; inactive modes are ignored.
"""
import math

import numpy as np

import oracle
import synth
from synth.fc3 import random_fc3

KB = 1.380649e-23
HBAR_KB = 6.62607015e-34 / (2.0 * math.pi) / KB * 1e12   # K ps


def _toy(w, v, r, a, T):
    omega = np.full((1, 3), w)
    vel = np.zeros((1, 3, 3))
    for j in range(3):
        vel[0, j, j] = v
    rates = np.full((len(T), 3), r)
    A = np.eye(3) * a
    return oracle.kappa_rta((1, 1, 1), 1, omega, vel, A, T, rates, np.zeros_like(rates))


def test_si_closed_form_and_classical_limit():
    w, v, r, a = 7.5, 42.0, 0.37, 3.1
    T = np.array([30.0, 300.0, 3000.0, 3.0e6])
    k, nskip = _toy(w, v, r, a, T)
    assert np.all(nskip == 0)
    for t, TT in enumerate(T):
        x = HBAR_KB * w / TT
        E = x * x * np.exp(x) / np.expm1(x) ** 2
        ref = KB * E * (v * 100.0) ** 2 * (1e-12 / r) / (a ** 3 * 1e-30)
        np.testing.assert_allclose(np.diag(k[t]), ref, rtol=1e-13)
        assert np.all(k[t][~np.eye(3, dtype=bool)] == 0.0)
    # classical limit: E -> 1
    classical = KB * (v * 100.0) ** 2 * (1e-12 / r) / (a ** 3 * 1e-30)
    assert abs(k[-1, 0, 0] / classical - 1.0) < 1e-9


def test_matthiessen_rule_and_scaling():
    inst = synth.small()
    rng = np.random.default_rng(4)
    T = [300.0, 700.0]
    tot = rng.uniform(0.1, 2.0, (2, inst.nmodes))
    f = rng.uniform(0.0, 1.0, (2, inst.nmodes))
    k1, _ = oracle.kappa_rta(inst.grid, 2, inst.omega, inst.vel, inst.cr.A, T, tot * f, tot * (1 - f))
    k2, _ = oracle.kappa_rta(inst.grid, 2, inst.omega, inst.vel, inst.cr.A, T, tot, 0 * tot)
    k3, _ = oracle.kappa_rta(inst.grid, 2, inst.omega, inst.vel, inst.cr.A, T, 2 * tot, 0 * tot)
    scale = np.abs(k2).max()
    assert np.max(np.abs(k1 - k2)) <= 1e-13 * scale
    assert np.max(np.abs(2.0 * k3 - k2)) <= 1e-13 * scale


def test_skipped_modes():
    inst = synth.small()
    T = [300.0]
    r = np.ones((1, inst.nmodes))
    r[0, 10] = 0.0                      # an active mode without scattering
    k, nskip = oracle.kappa_rta(inst.grid, 2, inst.omega, inst.vel, inst.cr.A, T, r, 0 * r)
    assert nskip[0] == 1
    r2 = r.copy()
    r2[0, 10] = 1e300                   # the same mode with negligible relaxation time
    k2, nskip2 = oracle.kappa_rta(inst.grid, 2, inst.omega, inst.vel, inst.cr.A, T, r2, 0 * r2)
    assert nskip2[0] == 0
    np.testing.assert_allclose(k, k2, rtol=1e-14, atol=1e-14 * np.abs(k).max())


def test_cubic_isotropy_diamond():
    inst = synth.small()
    m = oracle.Model.from_instance(inst)
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    fc3 = random_fc3(inst.cr, 3.0, np.random.default_rng(7))
    T = [300.0, 600.0]
    r4, _, _ = oracle.rates4(m, T, 1.0, 7, dq)
    r3, _ = oracle.rates3(m, fc3, T, 1.0, dq)
    k, nskip = oracle.kappa_rta(inst.grid, 2, inst.omega, inst.vel, inst.cr.A, T, r3, r4)
    assert np.all(nskip == 0)
    for t in range(len(T)):
        k0 = np.trace(k[t]) / 3.0
        assert k0 > 0
        assert np.max(np.abs(k[t] - k0 * np.eye(3))) <= 1e-12 * k0
    # four-phonon scattering lowers the conductivity
    k3only, _ = oracle.kappa_rta(inst.grid, 2, inst.omega, inst.vel, inst.cr.A, T, r3, 0 * r4)
    assert np.all(np.trace(k, axis1=1, axis2=2) < np.trace(k3only, axis1=1, axis2=2))
