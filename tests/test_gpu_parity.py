"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: kept-process counts bit-exact (the window predicate is FP64 in a fixed order on both
sides); FP64 rates within 1e-10 relative; FP32-contraction rates within 1e-4 relative.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from synth.crystal import grid_points, flat_index, minus_index

pytestmark = pytest.mark.gpu

RTOL64 = 1e-10
RTOL32 = 1e-4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fp4():
    import paper_2104_04895_amd as m
    return m


def _ctx(fp4, inst, **kw):
    c = fp4.Context(0)
    c.load_instance(inst, dq=oracle.default_dq(inst.cr.A, inst.grid), **kw)
    return c


def _oracle(inst, T, sb, mask, targets=None, want_rates=True, phi_scale=1.0):
    m = oracle.Model.from_instance(inst, phi_scale=phi_scale)
    return oracle.rates4(m, T, sb, mask, oracle.default_dq(inst.cr.A, inst.grid), targets,
                         want_rates=want_rates)


def _rel(a, b):
    den = np.maximum(np.abs(b), 1e-300)
    return np.max(np.where(b == 0, np.abs(a), np.abs(a - b) / den))


@pytest.fixture(scope="module")
def small():
    return synth.small()


def test_small_fp64_all_modes(fp4, small):
    """3x3x3 diamond, first-shell FC4, 300 K, all 162 modes: counts exact, rates 1e-10."""
    _say("case: small 3x3x3 fp64 all modes")
    r_o, rch_o, c_o = _oracle(small, small.T, 1.0, 7)
    with _ctx(fp4, small) as c:
        r, rch, cnt = c.compute_rates4(small.T, 1.0, 7, fp4.FP4_FP64, by_channel=True)
    assert np.array_equal(cnt, c_o)
    assert _rel(r, r_o) <= RTOL64
    assert _rel(rch, rch_o) <= RTOL64
    assert np.all(r[0, :3] == 0.0)


def test_small_fp32_contraction(fp4, small):
    """Same workload with the complex-FP32 contraction: identical counts, rates 1e-4."""
    _say("case: small 3x3x3 fp32")
    r_o, _, c_o = _oracle(small, small.T, 1.0, 7)
    with _ctx(fp4, small) as c:
        r, _, cnt = c.compute_rates4(small.T, 1.0, 7, fp4.FP4_FP32)
    assert np.array_equal(cnt, c_o)
    err = _rel(r, r_o)
    _say("fp32 max rel err", err)
    assert err <= RTOL32


@pytest.mark.parametrize("grid,rc,sb,mask,T", [
    ((3, 2, 4), synth.configs.RC_SECOND, 0.8, 7, (250.0, 600.0, 1200.0)),
    ((2, 2, 2), synth.configs.RC_SECOND, 1.3, 5, (300.0,)),
    ((5, 1, 1), synth.configs.RC_FIRST, 1.0, 2, (300.0, 700.0)),
    ((1, 1, 1), synth.configs.RC_SECOND, 1.0, 7, (300.0,)),
    ((3, 3, 3), synth.configs.RC_SECOND, 0.1, 7, (300.0,)),
    ((2, 3, 2), synth.configs.RC_FIRST, 1.0, 7,
     (100.0, 200.0, 300.0, 400.0, 600.0, 800.0, 1000.0, 1200.0)),
])
def test_ragged_grids_second_shell(fp4, grid, rc, sb, mask, T):
    """Non-cubic and degenerate grids, second-shell FC4 (1522 quartets, 34 groups), several
    temperatures (up to the maximum of 8) and channel masks, scalebroad down to 0.1 (the
    paper's setting, where the sigma floor fires more often); sampled targets for the
    oracle."""
    _say("case: ragged", grid, rc, sb, mask, T)
    inst = synth.diamond_instance(grid, rc, seed=31, T=T)
    rng = np.random.default_rng(1)
    nm = inst.nmodes
    targets = np.unique(np.concatenate([[0, nm - 1], rng.choice(nm, min(nm, 10), replace=False)]))
    r_o, rch_o, c_o = _oracle(inst, T, sb, mask, targets)
    with _ctx(fp4, inst) as c:
        r, rch, cnt = c.compute_rates4(T, sb, mask, fp4.FP4_FP64, targets=targets, by_channel=True)
        rall, _, call = c.compute_rates4(T, sb, mask, fp4.FP4_FP64)
    assert np.array_equal(cnt, c_o)
    assert _rel(r, r_o) <= RTOL64
    assert _rel(rch, rch_o) <= RTOL64
    # the subset entry point and the full-grid entry point agree bit for bit
    assert np.array_equal(rall[:, targets], r)
    assert np.array_equal(call[targets], cnt)


def test_ragged_tail_small_segments(fp4):
    """A 7x6x8 grid (336 points: the redistribution queueing takes two rounds of 256 points,
    the second ragged) with the smallest queue and list segments (64 and 64: one round per
    queue segment, the ++/-- scans flushed many times, lists evaluated in many passes):
    counts equal and FP64 rates within 1e-12 of the default segments', FP32 counts equal;
    the oracle's counts exact on 32 sampled modes and its rates on three (FP64 1e-10, FP32
    1e-4).  First-shell FC4 keeps the oracle's rates to a few seconds."""
    _say("case: ragged tail, small segments")
    inst = synth.diamond_instance((7, 6, 8), synth.configs.RC_FIRST, seed=41, T=(300.0, 800.0))
    nm = inst.nmodes
    rng = np.random.default_rng(4)
    tc = np.unique(np.concatenate([[3, nm - 1], rng.choice(nm, 30, replace=False)]))
    tr = np.array([3, nm // 2, nm - 1])
    with _ctx(fp4, inst) as c:
        r_d, _, c_d = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)
        c.set_param(fp4.FP4_PARAM_QSEG, 64)
        c.set_param(fp4.FP4_PARAM_LSEG, 64)
        r_s, _, c_s = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)
        r32, _, c32 = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP32)
    assert c_d.sum() > 0
    assert np.array_equal(c_s, c_d) and np.array_equal(c32, c_d)
    assert _rel(r_s, r_d) <= 1e-12
    _, _, c_o = _oracle(inst, inst.T, 1.0, 7, tc, want_rates=False)
    assert np.array_equal(c_d[tc], c_o)
    r_o, _, c_o3 = _oracle(inst, inst.T, 1.0, 7, tr)
    assert np.array_equal(c_d[tr], c_o3)
    assert _rel(r_d[:, tr], r_o) <= RTOL64
    assert _rel(r32[:, tr], r_o) <= RTOL32


def test_debug_matrix_elements(fp4):
    """V through the library's own contraction (W'', F, E3 F E4^T) against Eq. V4 evaluated
    literally by the oracle, all three channels, Umklapp included."""
    _say("case: debug V")
    inst = synth.diamond_instance((4, 4, 4), synth.configs.RC_SECOND, seed=7)
    m = oracle.Model.from_instance(inst)
    rng = np.random.default_rng(2)
    pts = grid_points(inst.grid)
    quads, modes, signs = [], [], []
    for _ in range(60):
        ch = int(rng.integers(0, 3))
        s1, s2 = [(1, 1), (1, -1), (-1, -1)][ch]
        iq, iq1, iq2 = (int(x) for x in rng.integers(0, inst.nq, 3))
        j, j1, j2, j3 = (int(x) for x in rng.integers(0, inst.nb, 4))
        iq3 = int(flat_index((pts[iq] + s1 * pts[iq1] + s2 * pts[iq2]) % np.asarray(inst.grid), inst.grid))
        quads.append([iq, j, iq1, j1, iq2, j2, j3, ch])
        modes.append([iq * 6 + j, iq1 * 6 + j1, iq2 * 6 + j2, iq3 * 6 + j3])
        signs.append([1, s1, s2, -1])
    V_o = oracle.v4(m, np.array(modes), np.array(signs))
    with _ctx(fp4, inst) as c:
        V64 = c.debug_matrix_elements(np.array(quads), fp4.FP4_FP64)
        V32 = c.debug_matrix_elements(np.array(quads), fp4.FP4_FP32)
    scale = np.max(np.abs(V_o))
    assert np.max(np.abs(V64 - V_o)) <= 1e-12 * scale
    assert np.max(np.abs(V32 - V_o)) <= 1e-5 * scale


def test_closed_form_gamma_only(fp4):
    """One atom at Gamma only (N = 1), hand-built modes: the HIP path reproduces the oracle
    (which is pinned to the hand-enumerated closed form)."""
    _say("case: gamma only")
    import itertools
    rng = np.random.default_rng(9)
    C = rng.standard_normal((3, 3, 3, 3))
    C = sum(np.transpose(C, p) for p in itertools.permutations(range(4))) / 24.0
    w = np.array([[10.0, 20.0, 30.0]])
    evec = np.zeros((1, 3, 1, 3), dtype=complex)
    for j in range(3):
        evec[0, j, 0, j] = 1.0
    vel = np.zeros((1, 3, 3))
    atoms = np.zeros((1, 4), dtype=np.int32)
    cells = np.zeros((1, 3, 3), dtype=np.int32)
    A = np.eye(3) * 3.0
    mo = oracle.Model((1, 1, 1), [12.0], w, evec, vel, atoms, cells, C.reshape(1, 81))
    r_o, _, c_o = oracle.rates4(mo, [400.0], 1.0, 7, 0.3)
    with fp4.Context(0) as c:
        c.load_lattice(A, (1, 1, 1), [12.0], 0.3)
        c.load_modes(w, evec, vel)
        c.load_fc4(atoms, cells, C.reshape(1, 81))
        r, _, cnt = c.compute_rates4([400.0], 1.0, 7, fp4.FP4_FP64)
    assert np.array_equal(cnt, c_o)
    assert _rel(r, r_o) <= RTOL64


def test_flat_bands_zero_velocity(fp4):
    """Dispersionless branches (10, 20, 30 rad/ps at every q) with zero group velocity on a
    2x2x2 grid: the window keeps exactly the processes with dw = 0 (e.g. 10 + 10 + 10 - 30),
    which sit on the edge of every frequency bound the kernel applies (row cull, sorted
    q'' scan).  Counts must equal the oracle's and rates agree to 1e-10."""
    _say("case: flat bands, zero velocity, 2x2x2")
    import itertools
    rng = np.random.default_rng(11)
    C = rng.standard_normal((3, 3, 3, 3))
    C = sum(np.transpose(C, p) for p in itertools.permutations(range(4))) / 24.0
    nq = 8
    w = np.tile(np.array([10.0, 20.0, 30.0]), (nq, 1))
    evec = np.zeros((nq, 3, 1, 3), dtype=complex)
    for j in range(3):
        evec[:, j, 0, j] = 1.0
    vel = np.zeros((nq, 3, 3))
    atoms = np.zeros((1, 4), dtype=np.int32)
    cells = np.zeros((1, 3, 3), dtype=np.int32)
    A = np.eye(3) * 3.0
    mo = oracle.Model((2, 2, 2), [12.0], w, evec, vel, atoms, cells, C.reshape(1, 81))
    r_o, _, c_o = oracle.rates4(mo, [300.0, 900.0], 1.0, 7, 0.3)
    with fp4.Context(0) as c:
        c.load_lattice(A, (2, 2, 2), [12.0], 0.3)
        c.load_modes(w, evec, vel)
        c.load_fc4(atoms, cells, C.reshape(1, 81))
        r, _, cnt = c.compute_rates4([300.0, 900.0], 1.0, 7, fp4.FP4_FP64)
        r32, _, cnt32 = c.compute_rates4([300.0, 900.0], 1.0, 7, fp4.FP4_FP32)
    assert c_o.sum() > 0 and c_o[:, 0].sum() > 0 and c_o[:, 2].sum() > 0
    assert np.array_equal(cnt, c_o) and np.array_equal(cnt32, c_o)
    assert _rel(r, r_o) <= RTOL64
    assert _rel(r32, r_o) <= RTOL32


def test_async_on_caller_stream(fp4, small):
    """fp4_compute_rates4_async on a torch stream into torch device tensors, as the first call
    after the loads (the per-q tables are built inside it) and again at other temperatures:
    identical to the synchronous call, channel rates summing to the total."""
    import torch
    _say("case: async entry point on a caller stream")
    nm = small.nmodes
    dev = torch.device("cuda:0")
    st = torch.cuda.Stream(device=dev)
    out = []
    with _ctx(fp4, small) as c:
        for T in ([300.0], [150.0, 600.0, 1200.0]):
            d_r = torch.empty((len(T), nm), dtype=torch.float64, device=dev)
            d_ch = torch.empty((len(T), 3, nm), dtype=torch.float64, device=dev)
            d_n = torch.empty((nm, 3), dtype=torch.int64, device=dev)
            c.compute_rates4_async(T, 1.0, 7, fp4.FP4_FP64, st.cuda_stream, d_r.data_ptr(),
                                   d_ch.data_ptr(), d_n.data_ptr())
            st.synchronize()
            out.append((T, d_r.cpu().numpy(), d_ch.cpu().numpy(), d_n.cpu().numpy()))
    with _ctx(fp4, small) as c:
        for T, r, rch, n in out:
            r_s, rch_s, n_s = c.compute_rates4(T, 1.0, 7, fp4.FP4_FP64, by_channel=True)
            assert np.array_equal(n, n_s)
            assert np.array_equal(r, r_s) and np.array_equal(rch, rch_s)
            assert _rel(rch.sum(axis=1), r) <= 1e-12


def test_normal_umklapp_split(fp4):
    """Rates restricted to normal or Umklapp processes (FP4_PARAM_QCLASS) against the
    oracle's class sums on every mode of the 3x3x3 diamond workload and of a 4x3x2
    orthorhombic one-atom cell: counts exact, FP64 rates within 1e-10, FP32 within 1e-4; the
    two classes add up to the unrestricted call."""
    from synth import configs
    for inst in (synth.small(), configs.ortho()):
        _say(f"case: normal/Umklapp split, {inst.name}")
        m = oracle.Model.from_instance(inst)
        dq = oracle.default_dq(inst.cr.A, inst.grid)
        parts = []
        with _ctx(fp4, inst) as c:
            r_all, _, c_all = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)
            for cls in (1, 2):
                c.set_param(fp4.FP4_PARAM_QCLASS, cls)
                r, _, cnt = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)
                r32, _, cnt32 = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP32)
                r_o, _, c_o = oracle.rates4_class(m, inst.cr.A, cls, inst.T, 1.0, 7, dq)
                assert c_o.sum() > 0
                assert np.array_equal(cnt, c_o) and np.array_equal(cnt32, c_o)
                assert _rel(r, r_o) <= RTOL64
                assert _rel(r32, r_o) <= RTOL32
                parts.append((r, cnt))
            c.set_param(fp4.FP4_PARAM_QCLASS, 0)
            r_back, _, _ = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)
        assert np.array_equal(parts[0][1] + parts[1][1], c_all)
        assert _rel(parts[0][0] + parts[1][0], r_all) <= 1e-12
        assert np.array_equal(r_back, r_all)


def _lattice_rotations(cr):
    """Integer matrices M = A T A^-1 of the crystal's point-group operations acting on reduced
    q coordinates (q = B^T f with B = 2 pi inv(A)^T, so f' = A T inv(A) f)."""
    A = np.asarray(cr.A, dtype=np.float64)
    Ai = np.linalg.inv(A)
    mats = []
    for T, _ in cr.ops:
        M = A @ np.asarray(T) @ Ai
        Mi = np.rint(M)
        assert np.max(np.abs(M - Mi)) < 1e-8
        mats.append(Mi.astype(np.int32))
    return np.unique(np.array(mats).reshape(-1, 9), axis=0)


def _degenerate_average(r, omega, nb):
    out = r.copy()
    w = np.asarray(omega).reshape(-1, nb)
    for iq in range(w.shape[0]):
        j = 0
        while j < nb:
            e = j + 1
            while e < nb and abs(w[iq, e] - w[iq, j]) <= 1e-9 * max(abs(w[iq, j]), 1e-30):
                e += 1
            out[:, iq * nb + j:iq * nb + e] = r[:, iq * nb + j:iq * nb + e].mean(axis=1, keepdims=True)
            j = e
    return out


def test_irreducible_wedge(fp4, small):
    """fp4_compute_rates4_wedge with the 48 point-group matrices of the diamond structure: only
    the irreducible points of the 3x3x3 grid are computed, and every rate equals the oracle's
    full-grid rate averaged over degenerate branches (1e-10); a matrix that does not map a
    3x3x2 grid onto itself is rejected."""
    _say("case: irreducible wedge, 3x3x3 diamond")
    rots = _lattice_rotations(small.cr)
    assert len(rots) == 48
    r_o, _, _ = _oracle(small, small.T, 1.0, 7)
    ref = _degenerate_average(r_o, small.omega, small.nb)
    with _ctx(fp4, small) as c:
        r, cnt, nirr = c.compute_rates4_wedge(small.T, 1.0, 7, fp4.FP4_FP64, rots)
        r32, _, _ = c.compute_rates4_wedge(small.T, 1.0, 7, fp4.FP4_FP32, rots)
    assert 1 < nirr < small.nq
    assert _rel(r, ref) <= RTOL64
    assert _rel(r32, ref) <= RTOL32
    inst = synth.diamond_instance((3, 3, 2), synth.configs.RC_FIRST, 5)
    swap = np.array([[0, 0, 1], [0, 1, 0], [1, 0, 0]], dtype=np.int32).reshape(1, 9)
    with _ctx(fp4, inst) as c:
        T = np.array([300.0])
        out = np.zeros(inst.nmodes)
        rc = c.call("fp4_compute_rates4_wedge", T.ctypes.data, 1, 1.0, 7, 0, 1, swap.ctypes.data,
                    out.ctypes.data, None, None)
        assert rc == fp4.FP4_E_INVAL


def test_phase_spaces(fp4, small):
    """FP4_PARAM_PHASE_SPACE 1 (weighted WP4) and 2 (P4) against the oracle's phase-space
    sums on every mode of the 3x3x3 workload, FP64 and FP32 settings (no contraction runs, so
    both are FP64 sums): counts exact, values within 1e-10; back to rates afterwards."""
    _say("case: phase spaces, 3x3x3")
    m = oracle.Model.from_instance(small)
    dq = oracle.default_dq(small.cr.A, small.grid)
    T = [300.0, 900.0]
    with _ctx(fp4, small) as c:
        r0, _, _ = c.compute_rates4(T, 1.0, 7, fp4.FP4_FP64)
        for kind in (1, 2):
            c.set_param(fp4.FP4_PARAM_PHASE_SPACE, kind)
            v, _, cnt = c.compute_rates4(T, 1.0, 7, fp4.FP4_FP64)
            v32, _, cnt32 = c.compute_rates4(T, 1.0, 7, fp4.FP4_FP32)
            ref, _, cref = oracle.phase_space4(m, kind, T, 1.0, 7, dq)
            assert cref.sum() > 0
            assert np.array_equal(cnt, cref) and np.array_equal(cnt32, cref)
            assert _rel(v, ref) <= RTOL64 and _rel(v32, ref) <= RTOL64
        c.set_param(fp4.FP4_PARAM_PHASE_SPACE, 0)
        r1, _, _ = c.compute_rates4(T, 1.0, 7, fp4.FP4_FP64)
    assert np.array_equal(r0, r1)


def test_properties_on_gpu(fp4, small):
    """Invariants that hold at any size, checked on the HIP path itself: time reversal
    (counts equal, rates equal to rounding), mask additivity, exact x4 under Phi -> 2 Phi."""
    _say("case: gpu properties")
    mq = minus_index(small.grid)
    with _ctx(fp4, small) as c:
        r, rch, cnt = c.compute_rates4([300.0], 1.0, 7, fp4.FP4_FP64, by_channel=True)
        parts = [c.compute_rates4([300.0], 1.0, 1 << ch, fp4.FP4_FP64) for ch in range(3)]
    r = r[0].reshape(small.nq, small.nb)
    assert np.array_equal(cnt.reshape(small.nq, small.nb, 3), cnt.reshape(small.nq, small.nb, 3)[mq])
    np.testing.assert_allclose(r[mq], r, rtol=1e-13)
    for ch in range(3):
        np.testing.assert_allclose(parts[ch][0][0], rch[0, ch], rtol=1e-14)
        assert np.array_equal(parts[ch][2][:, ch], cnt[:, ch])
    with _ctx(fp4, small, phi_scale=2.0) as c:
        r2, _, cnt2 = c.compute_rates4([300.0], 1.0, 7, fp4.FP4_FP64)
    assert np.array_equal(cnt2.reshape(small.nq, small.nb, 3), cnt.reshape(small.nq, small.nb, 3))
    assert np.array_equal(r2[0].reshape(small.nq, small.nb), 4.0 * r)


def test_error_paths(fp4, small):
    """Documented error codes; the context stays usable afterwards."""
    _say("case: error paths")
    import ctypes
    with fp4.Context(0) as c:
        T = np.array([300.0])
        out = np.zeros(small.nmodes)
        P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        assert c.call("fp4_compute_rates4", P(T), 1, 1.0, 7, 0, P(out), None, None) == fp4.FP4_E_STATE
        c.load_instance(small)
        assert c.call("fp4_compute_rates4", P(T), 1, 1.0, 0, 0, P(out), None, None) == fp4.FP4_E_INVAL
        assert c.call("fp4_compute_rates4", P(T), 1, -1.0, 7, 0, P(out), None, None) == fp4.FP4_E_INVAL
        bad = np.array([-3.0])
        assert c.call("fp4_compute_rates4", P(bad), 1, 1.0, 7, 0, P(out), None, None) == fp4.FP4_E_INVAL
        assert c.call("fp4_compute_rates4", P(T), 1, 1.0, 7, 9, P(out), None, None) == fp4.FP4_E_UNSUPPORTED
        assert c.call("fp4_compute_rates4", P(T), 9, 1.0, 7, 0, P(out), None, None) == fp4.FP4_E_INVAL
        om = small.omega.copy()
        om[3, 2] = np.nan
        with pytest.raises(fp4.Fp4Error) as e:
            c.load_modes(om, small.evec, small.vel)
        assert e.value.code == fp4.FP4_E_INVAL
        at = small.fc4.atoms.copy()
        at[0, 2] = 5
        with pytest.raises(fp4.Fp4Error) as e:
            c.load_fc4(at, small.fc4.cells, small.fc4.phi)
        assert e.value.code == fp4.FP4_E_INVAL
        tg = np.array([0, small.nmodes], dtype=np.int32)
        with pytest.raises(fp4.Fp4Error):
            c.compute_rates4([300.0], targets=tg)
        # still usable
        r, _, cnt = c.compute_rates4([300.0], 1.0, 7, fp4.FP4_FP64, targets=[5])
        assert cnt.sum() > 0 and r[0, 0] > 0


def test_medium_full_size_sampled(fp4):
    """The 8x8x8 second-shell workload at full size, two temperatures, in the launch
    configuration the benchmark times: counts of 48 sampled modes bit-exact, complete rates
    of one mode against the oracle, the recombination and splitting channels of three more
    modes, FP32 within 1e-4 on the same modes, and time reversal on the whole grid."""
    _say("case: medium 8x8x8 full size")
    inst = synth.medium()
    rng = np.random.default_rng(4)
    sample = rng.choice(np.arange(3, inst.nmodes), 48, replace=False)
    with _ctx(fp4, inst) as c:
        r, rch, cnt = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64, by_channel=True)
        r32, _, cnt32 = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP32)
    assert np.array_equal(cnt32, cnt)
    _, _, c_o = _oracle(inst, inst.T, 1.0, 7, sample, want_rates=False)
    assert np.array_equal(cnt[sample], c_o)
    mq = minus_index(inst.grid)
    rr = r.reshape(len(inst.T), inst.nq, inst.nb)
    np.testing.assert_allclose(rr[:, mq], rr, rtol=1e-12)
    side = sample[:3]
    r_o, rch_o, _ = _oracle(inst, inst.T, 1.0, 5, side)
    assert _rel(rch[:, 0][:, side], rch_o[:, 0]) <= RTOL64
    assert _rel(rch[:, 2][:, side], rch_o[:, 2]) <= RTOL64
    one = sample[3:4]
    _say("oracle: one full mode of the 8x8x8 workload")
    r_o, _, _ = _oracle(inst, inst.T, 1.0, 7, one)
    assert _rel(r[:, one], r_o) <= RTOL64
    assert _rel(r32[:, one], r_o) <= RTOL32


def test_three_atom_cell(fp4):
    """Nine branches (the 3-atom instantiation of the kernels): a layered 3-atom cell on a
    2x2x3 grid with 2001 quartets, two temperatures: counts exact and rates within 1e-10 on
    sampled targets, FP32 within 1e-4."""
    _say("case: three-atom cell 2x2x3")
    from synth import configs
    inst = configs.three_atom(grid=(2, 2, 3))
    targets = np.arange(0, inst.nmodes, 5)
    r_o, _, c_o = _oracle(inst, inst.T, 1.0, 7, targets)
    with _ctx(fp4, inst) as c:
        r, _, cnt = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64, targets)
        r32, _, cnt32 = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP32, targets)
    assert c_o.sum() > 0
    assert np.array_equal(cnt, c_o) and np.array_equal(cnt32, c_o)
    assert _rel(r, r_o) <= RTOL64
    assert _rel(r32, r_o) <= RTOL32


def test_one_atom_cell(fp4):
    """Three branches (the 1-atom instantiation of the kernels, whose group tiles are sized by
    the shared column records rather than by the 3x3 block): an FCC one-atom cell on a 3x3x4
    grid, every mode, two temperatures: counts exact, rates within 1e-10, FP32 within 1e-4."""
    _say("case: one-atom FCC cell 3x3x4")
    from synth import configs
    inst = configs.one_atom(grid=(3, 3, 4))
    r_o, _, c_o = _oracle(inst, inst.T, 1.0, 7)
    with _ctx(fp4, inst) as c:
        r, _, cnt = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)
        r32, _, cnt32 = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP32)
    assert c_o.sum() > 0
    assert np.array_equal(cnt, c_o) and np.array_equal(cnt32, c_o)
    assert _rel(r, r_o) <= RTOL64
    assert _rel(r32, r_o) <= RTOL32


def test_large_grid_properties(fp4):
    """The 16x16x16 workload (24 576 modes, the largest benchmarked grid), where the oracle
    is out of reach per mode: properties that hold at any size on 32 sampled q points and
    their time-reversed partners (equal counts, rates equal to rounding), and the FP32
    contraction within 1e-4 of FP64 with identical counts."""
    _say("case: large 16x16x16 properties")
    inst = synth.large()
    rng = np.random.default_rng(9)
    qs = rng.choice(np.arange(1, inst.nq), 32, replace=False)
    mq = minus_index(inst.grid)
    t1 = (qs[:, None] * inst.nb + np.arange(inst.nb)[None, :]).reshape(-1)
    t2 = (mq[qs][:, None] * inst.nb + np.arange(inst.nb)[None, :]).reshape(-1)
    with _ctx(fp4, inst) as c:
        r1, _, c1 = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64, t1)
        r2, _, c2 = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64, t2)
        r32, _, c32 = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP32, t1)
    assert c1.sum() > 0
    assert np.array_equal(c1, c2) and np.array_equal(c32, c1)
    np.testing.assert_allclose(r2, r1, rtol=1e-12)
    assert _rel(r32, r1) <= RTOL32


def test_normal_umklapp_split_even_fcc_grid(fp4):
    """Normal / Umklapp classes on the even 4x4x4 diamond grid, whose L, X and W points sit on
    the zone boundary (equally short first-zone images, the tie reading of the split): every
    mode, both classes against the oracle's class sums (counts exact, FP64 1e-10, FP32 1e-4)."""
    _say("case: normal/Umklapp split, 4x4x4 diamond")
    inst = synth.diamond_instance((4, 4, 4), synth.configs.RC_FIRST, seed=12, T=(300.0, 800.0))
    m = oracle.Model.from_instance(inst)
    dq = oracle.default_dq(inst.cr.A, inst.grid)
    refs = [oracle.rates4_class(m, inst.cr.A, cls, inst.T, 1.0, 7, dq) for cls in (1, 2)]
    with _ctx(fp4, inst) as c:
        for cls in (1, 2):
            c.set_param(fp4.FP4_PARAM_QCLASS, cls)
            r, _, cnt = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP64)
            r32, _, cnt32 = c.compute_rates4(inst.T, 1.0, 7, fp4.FP4_FP32)
            r_o, _, c_o = refs[cls - 1]
            assert c_o.sum() > 0
            assert np.array_equal(cnt, c_o) and np.array_equal(cnt32, c_o)
            assert _rel(r, r_o) <= RTOL64
            assert _rel(r32, r_o) <= RTOL32
        # both classes from one pass (the QCLASS setting is ignored by this call)
        for prec, tol in ((fp4.FP4_FP64, RTOL64), (fp4.FP4_FP32, RTOL32)):
            r, rn, ru, cnt = c.compute_rates4_classes(inst.T, 1.0, 7, prec)
            assert np.array_equal(cnt, refs[0][2] + refs[1][2])
            assert _rel(rn, refs[0][0]) <= tol and _rel(ru, refs[1][0]) <= tol
            assert _rel(r, refs[0][0] + refs[1][0]) <= tol
            assert _rel(rn + ru, r) <= 1e-12


def test_asymmetric_quartet_list(fp4, small):
    """A quartet list that is not symmetric under the slot-3/slot-4 exchange (random noise
    added to 10 quartets): the redistribution matrix element is then not symmetric in
    lambda'' and lambda''', so the mirror-pair shortcut must be off.  Rates of every mode
    against Eq. V4 evaluated literally by the oracle, redistribution only and all channels."""
    _say("case: asymmetric quartet list, 3x3x3")
    rng = np.random.default_rng(21)
    phi = small.fc4.phi.copy()
    pick = rng.choice(phi.shape[0], 10, replace=False)
    phi[pick] += rng.standard_normal((10, 81)) * np.abs(phi).max()
    mo = oracle.Model(small.grid, small.cr.mass, small.omega, small.evec, small.vel,
                      small.fc4.atoms, small.fc4.cells, phi)
    dq = oracle.default_dq(small.cr.A, small.grid)
    with fp4.Context(0) as c:
        c.load_lattice(small.cr.A, small.grid, small.cr.mass, dq)
        c.load_modes(small.omega, small.evec, small.vel)
        c.load_fc4(small.fc4.atoms, small.fc4.cells, phi)
        for mask in (fp4.FP4_PM, 7):
            r_o, _, c_o = oracle.rates4(mo, small.T, 1.0, mask, dq)
            r, _, cnt = c.compute_rates4(small.T, 1.0, mask, fp4.FP4_FP64)
            r32, _, cnt32 = c.compute_rates4(small.T, 1.0, mask, fp4.FP4_FP32)
            assert np.array_equal(cnt, c_o) and np.array_equal(cnt32, c_o)
            assert _rel(r, r_o) <= RTOL64
            assert _rel(r32, r_o) <= RTOL32


def test_injected_allocation_failure(fp4, small, monkeypatch):
    """FP4_TEST_FAIL_ALLOC=k makes the k-th device allocation of a context fail: the load that
    hits it returns FP4_E_NOMEM with a message, the context stays usable, and repeating the
    load then gives the same rates as an undisturbed context."""
    _say("case: injected allocation failure")
    with _ctx(fp4, small) as c:
        ref, _, ref_c = c.compute_rates4(small.T, 1.0, 7, fp4.FP4_FP64)
    monkeypatch.setenv("FP4_TEST_FAIL_ALLOC", "3")
    with fp4.Context(0) as c:
        monkeypatch.delenv("FP4_TEST_FAIL_ALLOC")
        dq = oracle.default_dq(small.cr.A, small.grid)
        c.load_lattice(small.cr.A, small.grid, small.cr.mass, dq)      # allocation 1
        with pytest.raises(fp4.Fp4Error) as e:
            c.load_modes(small.omega, small.evec, small.vel)          # allocations 2, 3, 4
        assert e.value.code == fp4.FP4_E_NOMEM
        assert "FP4_TEST_FAIL_ALLOC" in str(e.value)
        c.load_modes(small.omega, small.evec, small.vel)
        c.load_fc4(small.fc4.atoms, small.fc4.cells, small.fc4.phi)
        r, _, cnt = c.compute_rates4(small.T, 1.0, 7, fp4.FP4_FP64)
    assert np.array_equal(cnt, ref_c)
    assert np.array_equal(r, ref)
