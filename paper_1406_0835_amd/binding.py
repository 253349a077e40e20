"""ctypes binding of include/ofdft.h.  Names follow the C ABI (ofdft_<name> -> <name>).

Only argument marshalling happens here; every step of the evaluation and the
minimisation runs in libofdft.so.  There is no fallback: a missing library or a
failing call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

OK = 0
E_ARG, E_GRID, E_NOT_CONVERGED, E_NONFINITE, E_DEVICE, E_STATE = -1, -2, -3, -4, -5, -6
TF, SGA, VWTF, VT84F, KST2, TW, APBEF = range(7)
XC_NONE, XC_PZ81, XC_KSDT = 0, 1, 2
LPP_GAUSS, LPP_HA = 0, 1
FP64, MIXED = 0, 1
CG, TN = 0, 1

FUNCTIONAL_NAMES = {"TF": TF, "SGA": SGA, "VWTF": VWTF, "VT84F": VT84F, "KST2": KST2, "TW": TW, "APBEF": APBEF}


# device allocator callbacks of ofdft_options: void* alloc(size_t, void*), void free_(void*, void*)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("functional", ctypes.c_int), ("mu_sga", ctypes.c_double), ("xc", ctypes.c_int),
                ("lpp", ctypes.c_int), ("lpp_rc", ctypes.c_double), ("lpp_A", ctypes.c_double),
                ("lpp_qc", ctypes.c_double), ("precision", ctypes.c_int), ("minimizer", ctypes.c_int),
                ("tol_energy", ctypes.c_double), ("tol_residual", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("cg_precond", ctypes.c_double),
                ("extrapolate", ctypes.c_int), ("alloc", ALLOC_FN), ("free_", FREE_FN),
                ("alloc_ctx", ctypes.c_void_p), ("graph_cg", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("evaluations", ctypes.c_int), ("converged", ctypes.c_int),
                ("F_total", ctypes.c_double), ("E_internal", ctypes.c_double), ("F_s", ctypes.c_double),
                ("TS_s", ctypes.c_double), ("E_xc", ctypes.c_double), ("E_H", ctypes.c_double),
                ("E_ext", ctypes.c_double), ("E_alphaZ", ctypes.c_double), ("E_ion", ctypes.c_double),
                ("N_e", ctypes.c_double), ("mu", ctypes.c_double), ("residual", ctypes.c_double),
                ("TS_xc", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class OFDFTError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"ofdft error {code}: {message}")
        self.code = code


_LIB = None


def library_path() -> str:
    return os.environ.get("OFDFT_LIBRARY", os.path.join(_HERE, "libofdft.so"))


def _share_torch_hip_runtime() -> None:
    """PyTorch for ROCm carries its own copy of the HIP runtime (same soname as the system's,
    but its own libraries ask for it under another name).  Loading PyTorch first makes the
    library bind to that copy, so the process has one HIP runtime: device pointers from
    PyTorch's allocator and its streams are then valid in the library.  Loaded the other way
    round, PyTorch would start a second runtime that sees no GPU."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def load_library() -> ctypes.CDLL:
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise OFDFTError(E_DEVICE, f"{path} not found: build it with python -m paper_1406_0835_amd.build")
    _share_torch_hip_runtime()
    lib = ctypes.CDLL(path)
    P, D, I = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.ofdft_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.ofdft_default_options.restype = None
    sigs = {
        "ofdft_create": [ctypes.POINTER(Options), ctypes.POINTER(P)],
        "ofdft_destroy": [P],
        "ofdft_set_cell": [P, dp, D, ip],
        "ofdft_set_ions": [P, I, dp, dp],
        "ofdft_set_temperature": [P, D],
        "ofdft_minimize_density": [P, ctypes.POINTER(Report)],
        "ofdft_free_energy_and_forces": [P, dp, dp, dp, dp],
        "ofdft_get_density": [P, dp],
        "ofdft_set_density": [P, dp],
        "ofdft_eval": [P, ctypes.POINTER(Report), dp],
        "ofdft_time_evals": [P, I, dp, I, ctypes.POINTER(ctypes.c_char_p), dp, ip],
        "ofdft_batch_minimize": [ctypes.POINTER(P), I, ctypes.POINTER(Report)],
        "ofdft_autotune": [P, I, ip],
        "ofdft_set_tiles": [P, ip],
        "ofdft_ewald": [dp, I, dp, dp, dp, dp, dp],
        "ofdft_stress": [P, dp],
        "ofdft_eval_noalloc": [P, P, P, ctypes.POINTER(Report)],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ofdft_last_error.argtypes = [P]
    lib.ofdft_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(lib, rc: int, ctx=None):
    if rc != OK:
        msg = lib.ofdft_last_error(ctx)
        raise OFDFTError(rc, (msg or b"").decode())


def ewald(lattice, positions, charges, forces: bool = True, stress: bool = False):
    """Ion-ion Ewald energy (hartree), forces (hartree/bohr) and, with stress=True, its
    stress-tensor term (3, 3, hartree/bohr^3) as a third result; host code, no device."""
    lib = load_library()
    lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1))
    z = np.ascontiguousarray(np.asarray(charges, dtype=np.float64).reshape(-1))
    if pos.size != 3 * z.size:
        raise OFDFTError(E_ARG, "positions must be (nat, 3) and charges (nat,)")
    E = ctypes.c_double()
    f = np.zeros(3 * z.size) if forces else None
    sig = np.zeros(9) if stress else None
    _check(lib, lib.ofdft_ewald(_dptr(lat), int(z.size), _dptr(pos), _dptr(z), ctypes.byref(E),
                                _dptr(f) if forces else None, _dptr(sig) if stress else None))
    if stress:
        return E.value, (f.reshape(-1, 3) if forces else None), sig.reshape(3, 3)
    return E.value, (f.reshape(-1, 3) if forces else None)


def default_options(**kw) -> Options:
    lib = load_library()
    o = Options()
    lib.ofdft_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "functional" and isinstance(v, str):
            v = FUNCTIONAL_NAMES[v]
        if k == "precision" and isinstance(v, str):
            v = {"fp64": FP64, "mixed": MIXED}[v.lower()]
        if k == "minimizer" and isinstance(v, str):
            v = {"cg": CG, "tn": TN}[v.lower()]
        if k == "xc" and isinstance(v, str):
            v = {"none": XC_NONE, "pz81": XC_PZ81, "ksdt": XC_KSDT}[v.lower()]
        if k == "lpp" and isinstance(v, str):
            v = {"gauss": LPP_GAUSS, "ha": LPP_HA}[v.lower()]
        setattr(o, k, v)
    return o


class Context:
    """One ofdft_ctx.  Methods mirror the C entry points."""

    def __init__(self, options: Optional[Options] = None, **kw):
        self._lib = load_library()
        opts = options if options is not None else default_options(**kw)
        h = ctypes.c_void_p()
        _check(self._lib, self._lib.ofdft_create(ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self.options = opts
        self.shape = None
        self.nat = 0

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.ofdft_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_cell(self, lattice, grid: Sequence[int], cell_scale: float = 1.0):
        lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
        g = (ctypes.c_int * 3)(*[int(x) for x in grid])
        _check(self._lib, self._lib.ofdft_set_cell(self._h, _dptr(lat), float(cell_scale), g), self._h)
        self.shape = tuple(int(x) for x in grid)

    def set_ions(self, positions, charges):
        pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1))
        z = np.ascontiguousarray(np.asarray(charges, dtype=np.float64).reshape(-1))
        if pos.size != 3 * z.size:
            raise OFDFTError(E_ARG, "positions must be (nat, 3) and charges (nat,)")
        _check(self._lib, self._lib.ofdft_set_ions(self._h, int(z.size), _dptr(pos), _dptr(z)), self._h)
        self.nat = int(z.size)

    def set_temperature(self, T_kelvin: float):
        _check(self._lib, self._lib.ofdft_set_temperature(self._h, float(T_kelvin)), self._h)

    def minimize_density(self, check: bool = True) -> Report:
        rep = Report()
        rc = self._lib.ofdft_minimize_density(self._h, ctypes.byref(rep))
        if check:
            _check(self._lib, rc, self._h)
        self.last_rc = rc
        return rep

    def free_energy_and_forces(self, forces: bool = True, pressure: bool = False):
        """(F_total, E_internal, forces (nat, 3) or None[, pressure]) from
        ofdft_free_energy_and_forces; the pressure is appended when asked for."""
        F = ctypes.c_double()
        E = ctypes.c_double()
        P = ctypes.c_double()
        f = np.zeros(3 * self.nat) if forces else None
        rc = self._lib.ofdft_free_energy_and_forces(self._h, ctypes.byref(F), ctypes.byref(E),
                                                    _dptr(f) if forces else None,
                                                    ctypes.byref(P) if pressure else None)
        _check(self._lib, rc, self._h)
        out = (F.value, E.value, (f.reshape(-1, 3) if forces else None))
        return out + (P.value,) if pressure else out

    def stress(self) -> np.ndarray:
        """Stress tensor (3, 3) in hartree/bohr^3 at the converged density."""
        sig = np.zeros(9)
        _check(self._lib, self._lib.ofdft_stress(self._h, _dptr(sig)), self._h)
        return sig.reshape(3, 3)

    def pressure(self) -> float:
        """Pressure (hartree/bohr^3), the pressure output of ofdft_free_energy_and_forces."""
        return self.free_energy_and_forces(forces=False, pressure=True)[3]

    def get_density(self) -> np.ndarray:
        out = np.zeros(int(np.prod(self.shape)))
        _check(self._lib, self._lib.ofdft_get_density(self._h, _dptr(out)), self._h)
        return out.reshape(self.shape)

    def set_density(self, phi):
        p = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1))
        _check(self._lib, self._lib.ofdft_set_density(self._h, _dptr(p)), self._h)

    def eval(self, potential: bool = False):
        rep = Report()
        pot = np.zeros(int(np.prod(self.shape))) if potential else None
        _check(self._lib, self._lib.ofdft_eval(self._h, ctypes.byref(rep), _dptr(pot) if potential else None),
               self._h)
        return (rep, pot.reshape(self.shape)) if potential else rep

    def eval_noalloc(self, phi_dev: int, v_dev: int) -> Report:
        """ofdft_eval_noalloc: one evaluation at the amplitude in device memory phi_dev
        (N doubles, as given), the potential into device memory v_dev (N doubles), with no
        allocation (intermediates in the library's static device scratch array)."""
        rep = Report()
        _check(self._lib, self._lib.ofdft_eval_noalloc(self._h, ctypes.c_void_p(int(phi_dev)),
                                                       ctypes.c_void_p(int(v_dev)), ctypes.byref(rep)), self._h)
        return rep

    def autotune(self, n_evals: int = 5):
        """Pick FFT tiles (tr, tc, rb) by timing; returns the chosen triple."""
        t = (ctypes.c_int * 3)()
        _check(self._lib, self._lib.ofdft_autotune(self._h, int(n_evals), t), self._h)
        return tuple(t)

    def set_tiles(self, tiles):
        t = (ctypes.c_int * 3)(*[int(x) for x in tiles])
        _check(self._lib, self._lib.ofdft_set_tiles(self._h, t), self._h)

    def time_evals(self, n_evals: int, max_kernels: int = 16):
        """(total device ms, [(kernel name, average ms per evaluation)]); max_kernels=0: total only."""
        total = ctypes.c_double()
        names = (ctypes.c_char_p * max(max_kernels, 1))()
        ms = (ctypes.c_double * max(max_kernels, 1))()
        nk = ctypes.c_int()
        _check(self._lib, self._lib.ofdft_time_evals(self._h, int(n_evals), ctypes.byref(total), max_kernels,
                                                     names, ms, ctypes.byref(nk)), self._h)
        return total.value, [(names[k].decode(), ms[k]) for k in range(nk.value)]


def batch_minimize(contexts: Sequence[Context]):
    lib = load_library()
    n = len(contexts)
    arr = (ctypes.c_void_p * n)(*[c._h.value for c in contexts])
    reps = (Report * n)()
    _check(lib, lib.ofdft_batch_minimize(arr, n, reps))
    return [reps[i] for i in range(n)]
