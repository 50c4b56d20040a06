"""GPU parity of the RTA thermal conductivity with three- and four-phonon scattering
(fp4_compute_kappa_rta, through the C ABI) against the FP64 oracle: the oracle's conductivity
from the oracle's own 3ph and 4ph rates.

Bar: kappa within 1e-10 of the largest diagonal element (FP64 contraction; the off-diagonal
elements of the cubic crystal are zero up to rounding, so they are compared on that scale);
the rates the library used within 1e-10 of the oracle's; FP32 contraction within 1e-4."""
import numpy as np
import pytest

import oracle
import synth
from synth.fc3 import random_fc3

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def test_kappa_rta_diamond():
    import paper_2104_04895_amd as fp4
    _say("case: kappa RTA, 3x3x3 diamond, first-shell FC3 and FC4, T = 300/600 K")
    inst = synth.small()
    fc3 = random_fc3(inst.cr, 3.0, np.random.default_rng(7))
    T = [300.0, 600.0]
    m = oracle.Model.from_instance(inst)
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    r4_o, _, _ = oracle.rates4(m, T, 1.0, 7, dq)
    r3_o, _ = oracle.rates3(m, fc3, T, 1.0, dq)
    k_o, ns_o = oracle.kappa_rta(inst.grid, 2, inst.omega, inst.vel, inst.cr.A, T, r3_o, r4_o)
    with fp4.Context(0) as c:
        c.load_instance(inst, dq=dq)
        c.load_fc3(fc3.atoms, fc3.cells, fc3.phi)
        k, ns, r3, r4 = c.compute_kappa_rta(T, 1.0, fp4.FP4_FP64)
        k32, _, _, _ = c.compute_kappa_rta(T, 1.0, fp4.FP4_FP32)
    assert np.array_equal(ns, ns_o)
    den = lambda a: np.maximum(np.abs(a), 1e-300)
    assert np.max(np.abs(r4 - r4_o) / den(r4_o)) <= 1e-10
    assert np.max(np.abs(r3 - r3_o) / den(r3_o)) <= 1e-10
    for t in range(len(T)):
        scale = np.max(np.abs(np.diag(k_o[t])))
        e64 = np.max(np.abs(k[t] - k_o[t])) / scale
        e32 = np.max(np.abs(k32[t] - k_o[t])) / scale
        _say(f"  T {T[t]} K: kappa_xx {k[t, 0, 0]:.6f} W/(m K), err FP64 {e64:.1e}, FP32 {e32:.1e}")
        assert e64 <= 1e-10
        assert e32 <= 1e-4
