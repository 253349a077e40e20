"""C-ABI contract checks that need no GPU: the library loads, exports every
function declared in include/ofdft.h, the ctypes structs match the C layout,
and invalid arguments are rejected before any device work."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1406_0835_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ofdft.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.library_path()):
        from paper_1406_0835_amd import build
        build.build()
    return B.load_library()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ofdft_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("ofdft_set_cell", "ofdft_set_ions", "ofdft_set_temperature", "ofdft_minimize_density",
              "ofdft_free_energy_and_forces", "ofdft_create", "ofdft_destroy", "ofdft_eval"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", B.library_path()], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ofdft_\w+)", out))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, missing
    for n in _declared_functions():
        assert hasattr(lib, n)


def test_struct_layout_matches_c(lib):
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "ofdft.h"
int main(void) {
  printf("%zu %zu\n", sizeof(ofdft_options), sizeof(ofdft_report));
  printf("%zu %zu %zu %zu\n", offsetof(ofdft_options, precision), offsetof(ofdft_options, tol_energy),
         offsetof(ofdft_options, device), offsetof(ofdft_options, stream));
  printf("%zu %zu %zu\n", offsetof(ofdft_report, F_total), offsetof(ofdft_report, mu),
         offsetof(ofdft_report, residual));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        vals = [int(x) for x in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    O, R = B.Options, B.Report
    assert vals[0] == ctypes.sizeof(O) and vals[1] == ctypes.sizeof(R)
    assert vals[2:6] == [O.precision.offset, O.tol_energy.offset, O.device.offset, O.stream.offset]
    assert vals[6:9] == [R.F_total.offset, R.mu.offset, R.residual.offset]


def test_default_options(lib):
    o = B.Options()
    lib.ofdft_default_options(ctypes.byref(o))
    assert o.functional == B.TF and o.xc == B.XC_PZ81 and o.lpp == B.LPP_GAUSS
    assert o.lpp_rc == 0.5 and o.precision == B.FP64 and o.minimizer == B.CG
    assert o.tol_energy == 1e-8 and o.max_iter == 1000 and abs(o.mu_sga - 5 / 27) < 1e-16


@pytest.mark.parametrize("field,value", [("functional", 9), ("xc", 3), ("lpp", 5), ("precision", 2),
                                         ("minimizer", 7), ("tol_energy", 0.0), ("max_iter", 0),
                                         ("lpp_rc", -1.0)])
def test_create_rejects_invalid_options_before_device(lib, field, value):
    o = B.Options()
    lib.ofdft_default_options(ctypes.byref(o))
    setattr(o, field, value)
    h = ctypes.c_void_p()
    rc = lib.ofdft_create(ctypes.byref(o), ctypes.byref(h))
    assert rc == B.E_ARG
    assert not h.value
    assert lib.ofdft_last_error(None)


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.ofdft_create(None, None) == B.E_ARG
    assert lib.ofdft_set_cell(None, None, 1.0, None) == B.E_ARG
    assert lib.ofdft_set_temperature(None, 1e4) == B.E_ARG
    assert lib.ofdft_minimize_density(None, None) == B.E_ARG
    assert lib.ofdft_free_energy_and_forces(None, None, None, None, None) == B.E_ARG
    assert lib.ofdft_destroy(None) == B.E_ARG
    assert lib.ofdft_batch_minimize(None, 1, None) == B.E_ARG
    assert b"null" in lib.ofdft_last_error(None).lower() or lib.ofdft_last_error(None)
    del h


def test_no_device_is_reported_not_faked(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    o = B.Options()
    lib.ofdft_default_options(ctypes.byref(o))
    h = ctypes.c_void_p()
    assert lib.ofdft_create(ctypes.byref(o), ctypes.byref(h)) == B.E_DEVICE
    with pytest.raises(B.OFDFTError):
        B.Context()


def test_extrapolate_option_is_validated(lib):
    o = B.default_options(extrapolate=3)
    h = ctypes.c_void_p()
    rc = lib.ofdft_create(ctypes.byref(o), ctypes.byref(h))
    assert rc == B.E_ARG
    assert b"extrapolate" in lib.ofdft_last_error(None)
    assert B.default_options().extrapolate == 0
