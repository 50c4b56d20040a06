"""Python binding of the MI355X four-phonon RTA rate library (libfp4.so, C ABI in
include/fp4.h).

Argument marshalling only: every step of the rate computation runs in the HIP kernels of
libfp4.so.  Importing works without the library; creating a Context raises if libfp4.so has
not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfp4.so")

FP4_OK = 0
FP4_E_INVAL = -1
FP4_E_STATE = -2
FP4_E_NOMEM = -3
FP4_E_DEVICE = -4
FP4_E_UNSUPPORTED = -5

FP4_FP64 = 0
FP4_FP32 = 1

FP4_PARAM_WINDOW_W = 1
FP4_PARAM_SIGMA_MIN = 2
FP4_PARAM_QCHUNK = 3
FP4_PARAM_PROFILE = 4
FP4_PARAM_QCLASS = 5
FP4_PARAM_PHASE_SPACE = 6
FP4_PARAM_QSEG = 7
FP4_PARAM_LSEG = 8

FP4_PP, FP4_PM, FP4_MM = 1, 2, 4

EXPORTED = [
    "fp4_create", "fp4_destroy", "fp4_load_lattice", "fp4_load_modes", "fp4_load_fc4",
    "fp4_set_param", "fp4_compute_rates4", "fp4_compute_rates4_subset",
    "fp4_compute_rates4_async", "fp4_debug_matrix_elements", "fp4_last_stats",
    "fp4_last_timing", "fp4_last_error", "fp4_strerror", "fp4_batch_create",
    "fp4_batch_destroy", "fp4_batch_add", "fp4_batch_compute", "fp4_batch_last_timing",
    "fp4_batch_last_error", "fp4_autotune", "fp4_mlp_create", "fp4_mlp_destroy",
    "fp4_mlp_last_error", "fp4_mlp_num_params", "fp4_mlp_get_params", "fp4_mlp_set_params",
    "fp4_mlp_loss_grad", "fp4_mlp_train", "fp4_mlp_predict", "fp4_load_fc3",
    "fp4_compute_rates3", "fp4_surrogate_features", "fp4_compute_rates4_wedge",
    "fp4_compute_rates4_classes", "fp4_compute_rates4_noalloc", "fp4_compute_kappa_rta",
    "fp4_probe_matrix_rates", "fp4_autotune_shapes",
]
FP4_NFEAT = 18

_lib = None


class Fp4Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def lib():
    """Load libfp4.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2104_04895_amd.build` (no CPU fallback exists)")
        # PyTorch ships its own HIP runtime.  Loading it first makes the library bind to that
        # same runtime; a second runtime loaded before torch initialises leaves torch without
        # devices, which breaks torch streams and tensors passed to the async entry point.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, i32, u32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
        L.fp4_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
        L.fp4_destroy.argtypes = [P]
        L.fp4_destroy.restype = None
        L.fp4_load_lattice.argtypes = [P, P, P, i32, P, f64]
        L.fp4_load_modes.argtypes = [P, i32, i32, P, P, P]
        L.fp4_load_fc4.argtypes = [P, i32, P, P, P]
        L.fp4_set_param.argtypes = [P, i32, f64]
        L.fp4_load_fc3.argtypes = [P, i32, P, P, P]
        L.fp4_compute_rates3.argtypes = [P, P, i32, f64, P, i32, P, P]
        L.fp4_surrogate_features.argtypes = [P, P, i32, f64, P, i32, P, P, P, P]
        L.fp4_compute_rates4.argtypes = [P, P, i32, f64, u32, i32, P, P, P]
        L.fp4_compute_rates4_subset.argtypes = [P, P, i32, f64, u32, i32, P, i32, P, P, P]
        L.fp4_compute_rates4_wedge.argtypes = [P, P, i32, f64, u32, i32, i32, P, P, P, P]
        L.fp4_compute_rates4_classes.argtypes = [P, P, i32, f64, u32, i32, P, i32, P, P, P, P]
        L.fp4_compute_kappa_rta.argtypes = [P, P, i32, f64, i32, P, P, P, P]
        L.fp4_probe_matrix_rates.argtypes = [i32, P]
        L.fp4_compute_rates4_async.argtypes = [P, P, i32, f64, u32, i32, P, P, P, P]
        L.fp4_compute_rates4_noalloc.argtypes = [P, P, i32, f64, u32, i32, P, P, P, P]
        L.fp4_debug_matrix_elements.argtypes = [P, i32, P, i32, P]
        L.fp4_last_stats.argtypes = [P, P, P, P]
        L.fp4_last_timing.argtypes = [P, P, P]
        L.fp4_last_error.argtypes = [P]
        L.fp4_last_error.restype = ctypes.c_char_p
        L.fp4_strerror.argtypes = [ctypes.c_int]
        L.fp4_strerror.restype = ctypes.c_char_p
        L.fp4_batch_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
        L.fp4_batch_destroy.argtypes = [P]
        L.fp4_batch_destroy.restype = None
        L.fp4_batch_add.argtypes = [P, P]
        L.fp4_batch_compute.argtypes = [P, P, i32, f64, u32, i32, P, P]
        L.fp4_batch_last_timing.argtypes = [P, P, P, P]
        L.fp4_batch_last_error.argtypes = [P]
        L.fp4_batch_last_error.restype = ctypes.c_char_p
        L.fp4_autotune.argtypes = [P, P, i32, f64, u32, i32, i32, P, P, P, i32, P]
        L.fp4_autotune_shapes.argtypes = [P, P, i32, f64, u32, i32, i32, P, P, P, i32, P]
        u64 = ctypes.c_uint64
        L.fp4_mlp_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, i32, i32, i32, u64]
        L.fp4_mlp_destroy.argtypes = [P]
        L.fp4_mlp_destroy.restype = None
        L.fp4_mlp_last_error.argtypes = [P]
        L.fp4_mlp_last_error.restype = ctypes.c_char_p
        L.fp4_mlp_num_params.argtypes = [P]
        L.fp4_mlp_num_params.restype = ctypes.c_int64
        L.fp4_mlp_get_params.argtypes = [P, P]
        L.fp4_mlp_set_params.argtypes = [P, P]
        L.fp4_mlp_loss_grad.argtypes = [P, P, P, i32, P, P]
        L.fp4_mlp_train.argtypes = [P, P, P, i32, i32, i32, ctypes.c_float, u64, P]
        L.fp4_mlp_predict.argtypes = [P, P, i32, i32, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Context:
    """One library context on one HIP device (wraps fp4_create / fp4_destroy)."""

    def __init__(self, device: int = 0):
        self._L = lib()
        h = ctypes.c_void_p()
        rc = self._L.fp4_create(ctypes.byref(h), int(device))
        if rc != FP4_OK:
            raise Fp4Error(rc, f"fp4_create failed: {self._L.fp4_strerror(rc).decode()}")
        self._h = h
        self.nq = self.nb = 0

    def close(self):
        if getattr(self, "_h", None):
            self._L.fp4_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc, what):
        if rc != FP4_OK:
            msg = self._L.fp4_last_error(self._h).decode()
            raise Fp4Error(rc, f"{what}: {msg}")

    def call(self, name, *args):
        """Raw ABI call returning the status code (for error-path tests)."""
        return getattr(self._L, name)(self._h, *args)

    # ------------------------------------------------------------------ loads
    def load_lattice(self, A, grid, mass, dq=0.0):
        A = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
        g = np.ascontiguousarray(grid, dtype=np.int32)
        m = np.ascontiguousarray(mass, dtype=np.float64)
        self._check(self._L.fp4_load_lattice(self._h, _p(A), _p(g), len(m), _p(m), float(dq)),
                    "fp4_load_lattice")
        self.nq = int(np.prod(g))
        self.nb = 3 * len(m)

    def load_modes(self, omega, evec, vel):
        om = np.ascontiguousarray(omega, dtype=np.float64)
        ev = np.ascontiguousarray(evec, dtype=np.complex128).view(np.float64)
        ve = np.ascontiguousarray(vel, dtype=np.float64)
        self._check(self._L.fp4_load_modes(self._h, om.shape[0], om.shape[1], _p(om), _p(ev), _p(ve)),
                    "fp4_load_modes")

    def load_fc4(self, atoms, cells, phi):
        at = np.ascontiguousarray(atoms, dtype=np.int32)
        cl = np.ascontiguousarray(cells, dtype=np.int32)
        ph = np.ascontiguousarray(phi, dtype=np.float64)
        self._check(self._L.fp4_load_fc4(self._h, at.shape[0], _p(at), _p(cl), _p(ph)), "fp4_load_fc4")

    def load_fc3(self, atoms, cells, phi):
        at = np.ascontiguousarray(atoms, dtype=np.int32)
        cl = np.ascontiguousarray(cells, dtype=np.int32)
        ph = np.ascontiguousarray(phi, dtype=np.float64)
        self._check(self._L.fp4_load_fc3(self._h, at.shape[0], _p(at), _p(cl), _p(ph)), "fp4_load_fc3")

    def compute_rates3(self, T, scalebroad=1.0, targets=None, counts=True):
        """Three-phonon rates (Eq. 3phgamma): (rates [nT][nt], counts [nt][2] or None)."""
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        if targets is None:
            nt = self.nq * self.nb
        else:
            targets = np.ascontiguousarray(targets, dtype=np.int32)
            nt = len(targets)
        rates = np.zeros((len(T), nt))
        cnt = np.zeros((nt, 2), dtype=np.int64) if counts else None
        rc = self._L.fp4_compute_rates3(self._h, _p(T), len(T), float(scalebroad), _p(targets),
                                        nt, _p(rates), _p(cnt))
        self._check(rc, "fp4_compute_rates3")
        return rates, cnt

    def surrogate_features(self, T, scalebroad=1.0, targets=None, shift=None, scale=None):
        """Surrogate input rows X [nT][nt][FP4_NFEAT] (float32) and the three-phonon rates
        [nT][nt] they were built from."""
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        if targets is None:
            nt = self.nq * self.nb
        else:
            targets = np.ascontiguousarray(targets, dtype=np.int32)
            nt = len(targets)
        X = np.zeros((len(T), nt, FP4_NFEAT), dtype=np.float32)
        r3 = np.zeros((len(T), nt))
        if shift is not None:
            shift = np.ascontiguousarray(shift, dtype=np.float32)
            scale = np.ascontiguousarray(scale, dtype=np.float32)
        rc = self._L.fp4_surrogate_features(self._h, _p(T), len(T), float(scalebroad), _p(targets),
                                            nt, _p(shift), _p(scale), _p(X), _p(r3))
        self._check(rc, "fp4_surrogate_features")
        return X, r3

    def load_instance(self, inst, dq=0.0, phi_scale=1.0):
        self.load_lattice(inst.cr.A, inst.grid, inst.cr.mass, dq)
        self.load_modes(inst.omega, inst.evec, inst.vel)
        self.load_fc4(inst.fc4.atoms, inst.fc4.cells, inst.fc4.phi * phi_scale)

    def set_param(self, key, value):
        self._check(self._L.fp4_set_param(self._h, int(key), float(value)), "fp4_set_param")

    # ------------------------------------------------------------------ compute
    def compute_rates4(self, T, scalebroad=1.0, mask=7, precision=FP4_FP64, targets=None,
                       by_channel=False, counts=True):
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        nT = len(T)
        if targets is None:
            nt = self.nq * self.nb
        else:
            targets = np.ascontiguousarray(targets, dtype=np.int32)
            nt = len(targets)
        rates = np.zeros((nT, nt))
        rch = np.zeros((nT, 3, nt)) if by_channel else None
        cnt = np.zeros((nt, 3), dtype=np.int64) if counts else None
        if targets is None:
            rc = self._L.fp4_compute_rates4(self._h, _p(T), nT, float(scalebroad), int(mask),
                                            int(precision), _p(rates), _p(rch), _p(cnt))
        else:
            rc = self._L.fp4_compute_rates4_subset(self._h, _p(T), nT, float(scalebroad),
                                                   int(mask), int(precision), _p(targets), nt,
                                                   _p(rates), _p(rch), _p(cnt))
        self._check(rc, "fp4_compute_rates4")
        return rates, rch, cnt

    def compute_kappa_rta(self, T, scalebroad=1.0, precision=FP4_FP64):
        """RTA conductivity with 3ph + 4ph rates.  Returns (kappa[nT][3][3] W/(m K),
        nskip[nT], rates3[nT][nmodes], rates4[nT][nmodes])."""
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        nm = self.nq * self.nb
        kappa = np.zeros((len(T), 3, 3))
        nskip = np.zeros(len(T), dtype=np.int64)
        r3 = np.zeros((len(T), nm))
        r4 = np.zeros((len(T), nm))
        self._check(self._L.fp4_compute_kappa_rta(self._h, _p(T), len(T), float(scalebroad),
                                                  int(precision), _p(kappa), _p(nskip), _p(r3),
                                                  _p(r4)), "fp4_compute_kappa_rta")
        return kappa, nskip, r3, r4

    def compute_rates4_classes(self, T, scalebroad=1.0, mask=7, precision=FP4_FP64,
                               targets=None, counts=True):
        """Total, normal and Umklapp rates from one pass.  Returns (rates, normal, umklapp,
        counts), the rate arrays [nT][nt]."""
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        if targets is None:
            nt = self.nq * self.nb
        else:
            targets = np.ascontiguousarray(targets, dtype=np.int32)
            nt = len(targets)
        r, rn, ru = (np.zeros((len(T), nt)) for _ in range(3))
        cnt = np.zeros((nt, 3), dtype=np.int64) if counts else None
        self._check(self._L.fp4_compute_rates4_classes(self._h, _p(T), len(T), float(scalebroad),
                                                       int(mask), int(precision), _p(targets), nt,
                                                       _p(r), _p(rn), _p(ru), _p(cnt)),
                    "fp4_compute_rates4_classes")
        return r, rn, ru, cnt

    def compute_rates4_wedge(self, T, scalebroad, mask, precision, rotations, counts=True):
        """Rates on the irreducible grid points under integer rotations (reduced q
        coordinates), averaged over degenerate branches and copied to every equivalent point.
        Returns (rates[nT][nq*nb], counts[nq*nb][3] or None, number of irreducible points)."""
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        R = np.ascontiguousarray(rotations, dtype=np.int32).reshape(-1, 9)
        nm = self.nq * self.nb
        rates = np.zeros((len(T), nm))
        cnt = np.zeros((nm, 3), dtype=np.int64) if counts else None
        nirr = ctypes.c_int32()
        self._check(self._L.fp4_compute_rates4_wedge(self._h, _p(T), len(T), float(scalebroad),
                                                     int(mask), int(precision), len(R), _p(R),
                                                     _p(rates), _p(cnt), ctypes.byref(nirr)),
                    "fp4_compute_rates4_wedge")
        return rates, cnt, nirr.value

    def compute_rates4_async(self, T, scalebroad, mask, precision, stream_ptr, d_rates,
                             d_rates_ch=0, d_counts=0):
        """Device-pointer form (torch tensors' data_ptr() and a stream handle)."""
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        rc = self._L.fp4_compute_rates4_async(self._h, _p(T), len(T), float(scalebroad), int(mask),
                                              int(precision), ctypes.c_void_p(stream_ptr),
                                              ctypes.c_void_p(d_rates),
                                              ctypes.c_void_p(d_rates_ch or None),
                                              ctypes.c_void_p(d_counts or None))
        self._check(rc, "fp4_compute_rates4_async")

    def compute_rates4_noalloc(self, T, scalebroad, mask, precision, stream_ptr, d_rates,
                               d_rates_ch=0, d_counts=0):
        """Allocation-free device-pointer form (the library's fixed scratch area)."""
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        rc = self._L.fp4_compute_rates4_noalloc(self._h, _p(T), len(T), float(scalebroad),
                                                int(mask), int(precision),
                                                ctypes.c_void_p(stream_ptr),
                                                ctypes.c_void_p(d_rates),
                                                ctypes.c_void_p(d_rates_ch or None),
                                                ctypes.c_void_p(d_counts or None))
        self._check(rc, "fp4_compute_rates4_noalloc")

    def debug_matrix_elements(self, quads, precision=FP4_FP64):
        q = np.ascontiguousarray(quads, dtype=np.int32).reshape(-1, 8)
        V = np.zeros(len(q), dtype=np.complex128)
        self._check(self._L.fp4_debug_matrix_elements(self._h, len(q), _p(q), int(precision),
                                                      _p(V.view(np.float64))),
                    "fp4_debug_matrix_elements")
        return V

    def last_stats(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self._L.fp4_last_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
                    "fp4_last_stats")
        return {"processes": a.value, "candidates": b.value, "blocks": c.value}

    def last_timing(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self._L.fp4_last_timing(self._h, ctypes.byref(a), ctypes.byref(b)), "fp4_last_timing")
        return {"ms_main": a.value, "ms_total": b.value}


class Batch:
    """Several loaded Contexts evaluated by one captured HIP graph (fp4_batch_*)."""

    def __init__(self, device: int = 0):
        self._L = lib()
        h = ctypes.c_void_p()
        rc = self._L.fp4_batch_create(ctypes.byref(h), int(device))
        if rc != FP4_OK:
            raise Fp4Error(rc, "fp4_batch_create failed")
        self._h = h
        self.ctxs = []

    def close(self):
        if getattr(self, "_h", None):
            self._L.fp4_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc, what):
        if rc != FP4_OK:
            raise Fp4Error(rc, f"{what}: {self._L.fp4_batch_last_error(self._h).decode()}")

    def add(self, ctx: "Context"):
        self._check(self._L.fp4_batch_add(self._h, ctx._h), "fp4_batch_add")
        self.ctxs.append(ctx)

    def compute(self, T, scalebroad=1.0, mask=7, precision=FP4_FP64):
        """Returns ([rates_i [nT][nmodes_i]], [counts_i [nmodes_i][3]])."""
        T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
        sizes = [c.nq * c.nb for c in self.ctxs]
        rates = np.zeros(len(T) * sum(sizes))
        counts = np.zeros(3 * sum(sizes), dtype=np.int64)
        self._check(self._L.fp4_batch_compute(self._h, _p(T), len(T), float(scalebroad), int(mask),
                                              int(precision), _p(rates), _p(counts)),
                    "fp4_batch_compute")
        out_r, out_c, o_r, o_c = [], [], 0, 0
        for n in sizes:
            out_r.append(rates[o_r:o_r + len(T) * n].reshape(len(T), n))
            out_c.append(counts[o_c:o_c + 3 * n].reshape(n, 3))
            o_r += len(T) * n
            o_c += 3 * n
        return out_r, out_c

    def last_timing(self):
        ms, nb_, nl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self._L.fp4_batch_last_timing(self._h, ctypes.byref(ms), ctypes.byref(nb_),
                                                  ctypes.byref(nl)), "fp4_batch_last_timing")
        return {"ms_graph": ms.value, "graph_builds": nb_.value, "graph_launches": nl.value}


class Mlp:
    """The surrogate network (fp4_mlp_*): FP32 training and FP32/BF16 inference on the GPU."""

    def __init__(self, device: int = 0, nin: int = 10, width: int = 128, depth: int = 5,
                 seed: int = 0):
        self._L = lib()
        h = ctypes.c_void_p()
        rc = self._L.fp4_mlp_create(ctypes.byref(h), int(device), int(nin), int(width), int(depth),
                                    int(seed))
        if rc != FP4_OK:
            raise Fp4Error(rc, "fp4_mlp_create failed")
        self._h = h
        self.nin, self.width, self.depth = nin, width, depth
        self.nparam = int(self._L.fp4_mlp_num_params(h))

    def close(self):
        if getattr(self, "_h", None):
            self._L.fp4_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc, what):
        if rc != FP4_OK:
            raise Fp4Error(rc, f"{what}: {self._L.fp4_mlp_last_error(self._h).decode()}")

    def get_params(self):
        p = np.zeros(self.nparam, dtype=np.float32)
        self._check(self._L.fp4_mlp_get_params(self._h, _p(p)), "fp4_mlp_get_params")
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._check(self._L.fp4_mlp_set_params(self._h, _p(p)), "fp4_mlp_set_params")

    def loss_grad(self, X, y):
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        g = np.zeros(self.nparam, dtype=np.float32)
        L = ctypes.c_double()
        self._check(self._L.fp4_mlp_loss_grad(self._h, _p(X), _p(y), len(y), ctypes.byref(L), _p(g)),
                    "fp4_mlp_loss_grad")
        return L.value, g

    def train(self, X, y, epochs=10, batch=256, lr=1e-3, seed=0):
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        losses = np.zeros(epochs)
        self._check(self._L.fp4_mlp_train(self._h, _p(X), _p(y), len(y), int(epochs), int(batch),
                                          float(lr), int(seed), _p(losses)), "fp4_mlp_train")
        return losses

    def predict(self, X, bf16=True):
        X = np.ascontiguousarray(X, dtype=np.float32)
        out = np.zeros((len(X), 2), dtype=np.float32)
        ms = ctypes.c_double()
        self._check(self._L.fp4_mlp_predict(self._h, _p(X), len(X), 1 if bf16 else 0, _p(out),
                                            ctypes.byref(ms)), "fp4_mlp_predict")
        return out, ms.value


def autotune(ctx: "Context", T, scalebroad=1.0, mask=7, precision=FP4_FP64, nsample=64):
    """Run the q'-chunk autotuner on a context; returns (best, {qchunk: ms})."""
    L = lib()
    T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
    best = ctypes.c_int32()
    ms = np.zeros(16)
    qs = np.zeros(16, dtype=np.int32)
    n = ctypes.c_int32()
    ctx._check(L.fp4_autotune(ctx._h, _p(T), len(T), float(scalebroad), int(mask), int(precision),
                              int(nsample), ctypes.byref(best), _p(ms), _p(qs), 16, ctypes.byref(n)),
               "fp4_autotune")
    return best.value, {int(qs[i]): float(ms[i]) for i in range(n.value)}


def autotune_shapes(ctx: "Context", T, scalebroad=1.0, mask=7, precision=FP4_FP64, nsample=64):
    """Run the work-shape autotuner (q'-chunk, then queue and list segments); returns
    ((qchunk, qseg, lseg), [((qchunk, qseg, lseg), ms), ...])."""
    L = lib()
    T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
    best = np.zeros(3, dtype=np.int32)
    ms = np.zeros(32)
    cand = np.zeros((32, 3), dtype=np.int32)
    n = ctypes.c_int32()
    ctx._check(L.fp4_autotune_shapes(ctx._h, _p(T), len(T), float(scalebroad), int(mask),
                                     int(precision), int(nsample), _p(best), _p(ms), _p(cand), 32,
                                     ctypes.byref(n)), "fp4_autotune_shapes")
    return tuple(int(x) for x in best), [(tuple(int(x) for x in cand[i]), float(ms[i]))
                                         for i in range(min(n.value, 32))]


def probe_matrix_rates(device: int = 0) -> dict:
    """Measured TFLOP/s of the matrix cores and vector units (fp4_probe_matrix_rates)."""
    L = lib()
    t = np.zeros(6)
    rc = L.fp4_probe_matrix_rates(int(device), _p(t))
    if rc != FP4_OK:
        raise Fp4Error(rc, "fp4_probe_matrix_rates failed")
    keys = ["fp64_mfma_16x16x4", "fp64_valu_fma", "fp64_half_mfma_half_valu",
            "bf16_mfma_16x16x32", "fp32_valu_fma", "bf16_half_mfma_half_fp32_valu"]
    return dict(zip(keys, map(float, t)))
