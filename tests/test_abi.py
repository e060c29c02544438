"""The C-ABI library builds, loads and exports every symbol the header
declares; host-side argument checks reject bad calls before any device work
(these calls never reach the GPU, so they run on the CPU)."""
import ctypes
import subprocess

import pytest

import paper_1402_0264_amd as pm


@pytest.fixture(scope="module")
def L():
    return pm.lib()


def test_exports_every_declared_symbol(L):
    names = pm.declared_symbols()
    assert {"poly_mul_modp", "poly_mul_modp_async", "poly_divrem_modp", "poly_gcd_modp"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", pm.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)


def test_library_is_gfx950_only():
    import re
    blob = open(pm.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-z]+)", blob))
    assert targets == {b"gfx950"}


def _nf():
    return ctypes.c_int64(-7)


def test_host_checks_reject_bad_arguments(L):
    fake = 0x1000  # never dereferenced: every call below fails before device work
    nf = _nf()
    # non-prime and too-large moduli
    for p in (0, 1, 4, 469762051, 1 << 30, 2**31 - 1):
        st = L.poly_mul_modp(fake, 4, fake, 4, p, fake, 7, ctypes.byref(nf), None)
        assert st == pm.PM_EMODULUS, p
        assert "modulus" in pm.last_error()
    # capacity and lengths
    assert L.poly_mul_modp(fake, 4, fake, 4, 469762049, fake, 6, ctypes.byref(nf), None) == pm.PM_EINVAL
    assert L.poly_mul_modp(fake, -1, fake, 4, 469762049, fake, 9, ctypes.byref(nf), None) == pm.PM_EINVAL
    assert L.poly_mul_modp(None, 3, fake, 4, 469762049, fake, 9, ctypes.byref(nf), None) == pm.PM_EINVAL
    assert L.poly_mul_modp(fake, 4, fake, 4, 469762049, fake, 7, None, None) == pm.PM_EINVAL
    nq, nr = _nf(), _nf()
    assert L.poly_divrem_modp(fake, 5, fake, 0, 469762049, fake, 9, ctypes.byref(nq), fake, 9,
                              ctypes.byref(nr), None) == pm.PM_EDIVZERO
    assert L.poly_divrem_modp(fake, 9, fake, 3, 469762049, fake, 6, ctypes.byref(nq), fake, 9,
                              ctypes.byref(nr), None) == pm.PM_EINVAL
    assert L.poly_gcd_modp(fake, 5, fake, 5, 998244352, fake, 5, ctypes.byref(nf), None) == pm.PM_EMODULUS
    assert nf.value == -7 and nq.value == -7  # outputs untouched on failure


def test_params_roundtrip_and_validation():
    pm.set_params(mul_s=512, mul_r=8, div_s=16, gcd_s=32)
    assert pm.get_params() == {"mul_s": 512, "mul_r": 8, "div_s": 16, "gcd_s": 32, "mul_engine": 0}
    with pytest.raises(pm.PolyModPError):
        pm.set_params(mul_r=3)
    with pytest.raises(pm.PolyModPError):
        pm.set_params(gcd_s=1000)
    with pytest.raises(pm.PolyModPError):
        pm.set_params(mul_engine=3)
    pm.set_params(mul_engine=pm.MUL_MFMA)
    assert pm.get_params()["mul_engine"] == 2
    pm.set_params()
    assert pm.get_params() == {"mul_s": 0, "mul_r": 0, "div_s": 0, "gcd_s": 0, "mul_engine": 0}
