"""Python binding of the MI355X two-site shell-model DMRG library.

A thin ctypes layer over the C ABI in include/dmrg.h: it marshals arguments
and checks status codes; every step of the computation runs in the HIP
library `libdmrg_mi355x.so` built in-tree (see `build.py`).  Importing this
package does not load the library; the first `Context` does, and raises if
the built library is missing.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmrg_mi355x.so")

FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2

STATUS = {0: "OK", 1: "WARN_NOT_CONVERGED", -1: "ERR_ARG", -2: "ERR_HAMILTONIAN", -3: "ERR_TARGET",
          -4: "ERR_STATE", -5: "ERR_OUT_OF_MEMORY", -6: "ERR_DEVICE"}


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("davidson_tol", ctypes.c_double), ("davidson_max_iter", ctypes.c_int32),
                ("davidson_max_subspace", ctypes.c_int32), ("noise", ctypes.c_double),
                ("noise_sweeps", ctypes.c_int32), ("select_basis", ctypes.c_int32),
                ("tie_tol", ctypes.c_double), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("mem_cap_bytes", ctypes.c_uint64),
                ("scratch_bytes", ctypes.c_uint64), ("trunc_eps", ctypes.c_double),
                ("d_min", ctypes.c_int32), ("n_states", ctypes.c_int32),
                ("measure", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("group_products", ctypes.c_int32)]


class SweepStats(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("last_theta", ctypes.c_double),
                ("discarded_max", ctypes.c_double), ("discarded_sum", ctypes.c_double),
                ("products_low", ctypes.c_int64), ("products_fp64", ctypes.c_int64),
                ("solves", ctypes.c_int64), ("not_converged", ctypes.c_int64),
                ("heff_flops", ctypes.c_double), ("heff_seconds", ctypes.c_double),
                ("sweep_seconds", ctypes.c_double), ("renorm_seconds", ctypes.c_double),
                ("blocking_seconds", ctypes.c_double), ("density_seconds", ctypes.c_double),
                ("eig_seconds", ctypes.c_double), ("renormalize_seconds", ctypes.c_double),
                ("predict_seconds", ctypes.c_double), ("status", ctypes.c_int32),
                ("steps", ctypes.c_int32),
                ("gemm1_launches", ctypes.c_int64), ("gemm2_launches", ctypes.c_int64),
                ("gemm1_seconds", ctypes.c_double), ("gemm2_seconds", ctypes.c_double),
                ("gemm1_flops", ctypes.c_double), ("gemm2_flops", ctypes.c_double),
                ("gemm1_bytes", ctypes.c_double), ("gemm2_bytes", ctypes.c_double),
                ("reduce_seconds", ctypes.c_double), ("kept_max", ctypes.c_int64),
                ("energy_excited", ctypes.c_double), ("measure_seconds", ctypes.c_double),
                ("heff_flops_executed", ctypes.c_double),
                ("gemm1_issued_flops", ctypes.c_double), ("gemm2_issued_flops", ctypes.c_double),
                ("check_solves", ctypes.c_int64), ("check_max_rel", ctypes.c_double),
                ("delta_energy", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class DMRGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    """Attach the C signatures of include/dmrg.h to a loaded library."""
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "dmrg_default_options": (None, [ctypes.POINTER(Options)]),
        "dmrg_create": (I32, [ctypes.POINTER(Options), ctypes.POINTER(P)]),
        "dmrg_destroy": (None, [P]),
        "dmrg_load_hamiltonian": (I32, [P, I32, P, P, P, P, I32, I32, I32]),
        "dmrg_sweep": (I32, [P, P, I32, ctypes.POINTER(SweepStats)]),
        "dmrg_sweep_steps": (I32, [P, P, I32, I32, ctypes.POINTER(SweepStats)]),
        "dmrg_heff_layout": (I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I64), ctypes.POINTER(I32), P, P]),
        "dmrg_heff_apply": (I32, [P, P, P, I32]),
        "dmrg_check_fp64": (I32, [P, I32]),
        "dmrg_set_cideas": (I32, [P, P, P]),
        "dmrg_heff_apply_noalloc": (I32, [P, P, P, I32]),
        "dmrg_energy": (I32, [P, ctypes.POINTER(D)]),
        "dmrg_get_psi": (I32, [P, P]),
        "dmrg_heff_configs": (I32, [P, P]),
        "dmrg_sweep_many": (I32, [P, I32, P, P, P]),
        "dmrg_orbital_entropies": (I32, [P, P, P, P, P, P]),
        "dmrg_fiedler_ordering": (I32, [P, I32, P, ctypes.POINTER(D)]),
        "dmrg_status_string": (ctypes.c_char_p, [I32]),
        "dmrg_last_error": (ctypes.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib: Optional[ctypes.CDLL] = None


def library() -> ctypes.CDLL:
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python build.py` (hipcc, gfx950) first")
        # PyTorch ships its own HIP and HSA runtimes under other file names.  When
        # this library (and with it the system runtime) is loaded first and torch
        # afterwards, the library's device query finds no device; with torch
        # loaded first both runtimes work.  So load torch first when it exists.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        _lib = declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dev_ptr(x) -> int:
    """Device pointer of a torch tensor (float64, contiguous, on a GPU) or an int."""
    if isinstance(x, int):
        return x
    if x.dtype != __import__("torch").float64 or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("vectors must be contiguous float64 tensors on the GPU")
    return x.data_ptr()


class Context:
    """One DMRG context (one device, one stream)."""

    def __init__(self, lib: Optional[ctypes.CDLL] = None, **options):
        self._lib = lib if lib is not None else library()
        o = Options()
        self._lib.dmrg_default_options(ctypes.byref(o))
        for k, v in options.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        self.options = o
        h = ctypes.c_void_p()
        st = self._lib.dmrg_create(ctypes.byref(o), ctypes.byref(h))
        if st != 0:
            raise DMRGError(st, self._lib.dmrg_last_error(None).decode())
        self._h = h
        self.n_sites = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dmrg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, allow_warn: bool = True) -> int:
        if st < 0 or (st > 0 and not allow_warn):
            raise DMRGError(st, self._lib.dmrg_last_error(self._h).decode())
        return st

    def load_hamiltonian(self, species, two_m, eps, V, n_p: int, n_n: int, two_M: int) -> None:
        sp, tm, e, v = _i32(species), _i32(two_m), _f64(eps), _f64(V)
        n = sp.shape[0]
        if v.size != n ** 4:
            raise ValueError("V must have n_sites**4 elements")
        self._check(self._lib.dmrg_load_hamiltonian(self._h, n, _ptr(sp), _ptr(tm), _ptr(e), _ptr(v),
                                                    n_p, n_n, two_M))
        self.n_sites = n

    def _ord(self, ordering):
        if ordering is None:
            return None, None
        o = _i32(ordering)
        return o, _ptr(o)

    def sweep(self, D: int, ordering=None) -> dict:
        st = SweepStats()
        o, p = self._ord(ordering)
        code = self._check(self._lib.dmrg_sweep(self._h, p, D, ctypes.byref(st)))
        d = st.as_dict()
        d["code"] = code
        return d

    def sweep_steps(self, D: int, n_steps: int, ordering=None) -> dict:
        st = SweepStats()
        o, p = self._ord(ordering)
        code = self._check(self._lib.dmrg_sweep_steps(self._h, p, D, n_steps, ctypes.byref(st)))
        d = st.as_dict()
        d["code"] = code
        return d

    def heff_layout(self):
        bond, dim, ns = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        self._check(self._lib.dmrg_heff_layout(self._h, ctypes.byref(bond), ctypes.byref(dim),
                                               ctypes.byref(ns), None, None))
        qn = np.zeros((ns.value, 3), np.int32)
        dims = np.zeros((ns.value, 2), np.int64)
        self._check(self._lib.dmrg_heff_layout(self._h, ctypes.byref(bond), ctypes.byref(dim),
                                               ctypes.byref(ns), _ptr(qn), _ptr(dims)))
        return bond.value, dim.value, qn, dims

    def heff_apply(self, x, y, precision: int = FP64) -> None:
        """y = H_eff x on the context stream (device pointers or torch tensors)."""
        self._check(self._lib.dmrg_heff_apply(self._h, ctypes.c_void_p(_dev_ptr(x)),
                                              ctypes.c_void_p(_dev_ptr(y)), precision))

    def heff_apply_noalloc(self, x, y, precision: int = FP64) -> None:
        """y = H_eff x with the library's fixed device scratch (dmrg_heff_apply_noalloc)."""
        self._check(self._lib.dmrg_heff_apply_noalloc(self._h, ctypes.c_void_p(_dev_ptr(x)),
                                                      ctypes.c_void_p(_dev_ptr(y)), precision))

    def set_cideas(self, s1=None, n1=None) -> None:
        """CI-DEAS start from entropies and occupations (site indices) of a
        preprocessing run; both None: the hash start (dmrg_set_cideas)."""
        if s1 is None and n1 is None:
            self._check(self._lib.dmrg_set_cideas(self._h, None, None))
            return
        a, b = _f64(s1), _f64(n1)
        if a.size != self.n_sites or b.size != self.n_sites:
            raise ValueError("s1 and n1 need n_sites entries")
        self._check(self._lib.dmrg_set_cideas(self._h, _ptr(a), _ptr(b)))

    def check_fp64(self, on: bool) -> None:
        """Repeat every mixed-precision solve in FP64 from the same guess and
        report the largest energy difference (dmrg_check_fp64)."""
        self._check(self._lib.dmrg_check_fp64(self._h, 1 if on else 0))

    def energy(self) -> float:
        e = ctypes.c_double()
        self._check(self._lib.dmrg_energy(self._h, ctypes.byref(e)))
        return e.value

    def get_psi(self) -> np.ndarray:
        _, dim, _, _ = self.heff_layout()
        out = np.empty(dim, np.float64)
        self._check(self._lib.dmrg_get_psi(self._h, _ptr(out)))
        return out

    def heff_configs(self) -> np.ndarray:
        _, dim, _, _ = self.heff_layout()
        out = np.empty(dim, np.uint64)
        self._check(self._lib.dmrg_heff_configs(self._h, _ptr(out)))
        return out


    def orbital_entropies(self) -> dict:
        """Entropies and correlations of the last sweep run with measure=1
        (dmrg_orbital_entropies): s1[site], mutual[site, site'], n1, nn, hop."""
        n = self.n_sites
        out = {"s1": np.empty(n), "mutual": np.empty((n, n)), "n1": np.empty(n),
               "nn": np.empty((n, n)), "hop": np.empty((n, n))}
        self._check(self._lib.dmrg_orbital_entropies(self._h, *[_ptr(out[k]) for k in
                                                                ("s1", "mutual", "n1", "nn", "hop")]))
        return out


def fiedler_ordering(mutual, lib: Optional[ctypes.CDLL] = None):
    """(ordering, Fiedler value) of a mutual-information matrix (dmrg_fiedler_ordering)."""
    lib = lib if lib is not None else library()
    m = _f64(mutual)
    n = m.shape[0]
    if m.ndim != 2 or m.shape[1] != n:
        raise ValueError("mutual must be a square matrix")
    order = np.empty(n, np.int32)
    val = ctypes.c_double()
    st = lib.dmrg_fiedler_ordering(_ptr(m), n, _ptr(order), ctypes.byref(val))
    if st != 0:
        raise DMRGError(st, "dmrg_fiedler_ordering: n < 1 or a matrix that is not finite and symmetric")
    return order, val.value


def sweep_many(contexts, D, orderings=None):
    """One sweep of every context (dmrg_sweep_many); returns per-context stats."""
    lib = contexts[0]._lib
    n = len(contexts)
    handles = (ctypes.c_void_p * n)(*[c._h.value for c in contexts])
    Ds = _i32(D)
    stats = (SweepStats * n)()
    keep = []
    ords = None
    if orderings is not None:
        arrs = [None if o is None else _i32(o) for o in orderings]
        keep = arrs
        ords = (ctypes.c_void_p * n)(*[None if a is None else a.ctypes.data for a in arrs])
    st = lib.dmrg_sweep_many(handles, n, ords, _ptr(Ds), stats)
    del keep
    out = [s.as_dict() for s in stats]
    return st, out
