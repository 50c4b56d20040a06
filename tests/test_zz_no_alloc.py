"""GPU test of the allocation-free entry point fp4_compute_rates4_noalloc (called through the
C ABI) against the allocating fp4_compute_rates4_async on the same inputs: two calls in a row,
the second with a smaller input (so stale scratch contents of the first cannot leak into the
second), counts bit-exact and FP64 rates within 1e-10 (in practice identical), FP32 within
1e-4; a problem too large for the scratch area is rejected with FP4_E_UNSUPPORTED."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _run(fp4, inst, T, precision, noalloc):
    import torch
    dev = torch.device("cuda:0")
    st = torch.cuda.Stream(device=dev)
    nm = inst.nmodes
    d_r = torch.full((len(T), nm), -1.0, dtype=torch.float64, device=dev)
    d_ch = torch.full((len(T), 3, nm), -1.0, dtype=torch.float64, device=dev)
    d_n = torch.full((nm, 3), -1, dtype=torch.int64, device=dev)
    with fp4.Context(0) as c:
        c.load_instance(inst, dq=oracle.default_dq(inst.cr.A, inst.grid))
        f = c.compute_rates4_noalloc if noalloc else c.compute_rates4_async
        f(T, 1.0, 7, precision, st.cuda_stream, d_r.data_ptr(), d_ch.data_ptr(), d_n.data_ptr())
        st.synchronize()
    return d_r.cpu().numpy(), d_ch.cpu().numpy(), d_n.cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def test_noalloc_matches_async_two_calls():
    import paper_2104_04895_amd as fp4
    first = synth.diamond_instance((4, 4, 4), synth.configs.RC_SECOND, seed=5, T=(300.0, 900.0))
    second = synth.diamond_instance((3, 2, 2), synth.configs.RC_FIRST, seed=6, T=(500.0,))
    for inst in (first, second):
        for prec, tol in ((fp4.FP4_FP64, 1e-10), (fp4.FP4_FP32, 1e-4)):
            _say(f"case: noalloc vs async, {inst.name}, precision {prec}")
            ref = _run(fp4, inst, inst.T, prec, False)
            got = _run(fp4, inst, inst.T, prec, True)
            assert np.array_equal(got[2], ref[2])
            assert ref[2].sum() > 0
            e = max(_rel(got[0], ref[0]), _rel(got[1], ref[1]))
            _say(f"  max rel diff {e:.2e}, identical: {np.array_equal(got[0], ref[0])}")
            assert e <= tol


def test_noalloc_rejects_too_large():
    import ctypes
    import paper_2104_04895_amd as fp4
    import torch
    # 56x56x56 one-atom grid, 8 temperatures: the occupations alone (2 x 8 x 526 848
    # doubles) exceed the 64 MiB scratch area
    g = (56, 56, 56)
    nq = int(np.prod(g))
    w = np.zeros((nq, 3))
    ev = np.zeros((nq, 3, 1, 3), dtype=complex)
    for j in range(3):
        ev[:, j, 0, j] = 1.0
    with fp4.Context(0) as c:
        c.load_lattice(np.eye(3) * 3.0, g, [12.0], 0.3)
        c.load_modes(w, ev, np.zeros((nq, 3, 3)))
        c.load_fc4(np.zeros((1, 4), np.int32), np.zeros((1, 3, 3), np.int32), np.ones((1, 81)))
        T = np.linspace(100.0, 800.0, 8)
        d = torch.empty((8, nq * 3), dtype=torch.float64, device="cuda:0")
        rc = c._L.fp4_compute_rates4_noalloc(c._h, T.ctypes.data_as(ctypes.c_void_p), 8, 1.0, 7, 0,
                                             None, ctypes.c_void_p(d.data_ptr()), None, None)
        assert rc == fp4.FP4_E_UNSUPPORTED
        assert b"scratch" in c._L.fp4_last_error(c._h)
