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
    # never dereferenced: every call below fails before device work
    fa, fb, ff, fr = 0x10000, 0x20000, 0x30000, 0x40000
    nf = _nf()
    # non-prime and too-large moduli
    for p in (0, 1, 4, 469762051, 1 << 30, 2**31 - 1):
        st = L.poly_mul_modp(fa, 4, fb, 4, p, ff, 7, ctypes.byref(nf), None)
        assert st == pm.PM_EMODULUS, p
        assert "modulus" in pm.last_error()
    # capacity and lengths
    assert L.poly_mul_modp(fa, 4, fb, 4, 469762049, ff, 6, ctypes.byref(nf), None) == pm.PM_EINVAL
    assert L.poly_mul_modp(fa, -1, fb, 4, 469762049, ff, 9, ctypes.byref(nf), None) == pm.PM_EINVAL
    assert L.poly_mul_modp(None, 3, fb, 4, 469762049, ff, 9, ctypes.byref(nf), None) == pm.PM_EINVAL
    assert L.poly_mul_modp(fa, 4, fb, 4, 469762049, ff, 7, None, None) == pm.PM_EINVAL
    nq, nr = _nf(), _nf()
    assert L.poly_divrem_modp(fa, 5, fb, 0, 469762049, ff, 9, ctypes.byref(nq), fr, 9,
                              ctypes.byref(nr), None) == pm.PM_EDIVZERO
    assert L.poly_divrem_modp(fa, 9, fb, 3, 469762049, ff, 6, ctypes.byref(nq), fr, 9,
                              ctypes.byref(nr), None) == pm.PM_EINVAL
    assert L.poly_gcd_modp(fa, 5, fb, 5, 998244352, ff, 5, ctypes.byref(nf), None) == pm.PM_EMODULUS
    assert nf.value == -7 and nq.value == -7  # outputs untouched on failure


def test_outputs_overlapping_inputs_are_rejected(L):
    """Every entry point refuses an output that overlaps an input, or two
    outputs that overlap, with PM_EINVAL before any device work (the
    pointers are never dereferenced)."""
    p = 469762049
    a, b = 0x100000, 0x200000          # 16 words each
    i64 = ctypes.c_int64
    n1, n2, n3 = i64(-7), i64(-7), i64(-7)
    r = ctypes.byref

    def rejected(st):
        return st == pm.PM_EINVAL and "overlap" in pm.last_error()

    # f starting inside a, f running into b, f exactly on b
    for f in (a + 4 * 8, b - 4 * 4, b):
        assert rejected(L.poly_mul_modp(a, 16, b, 16, p, f, 31, r(n1), None)), hex(f)
        assert rejected(L.poly_mul_modp_async(a, 16, b, 16, p, f, 31, None, None, None))
        assert rejected(L.poly_mul_modp_noalloc(a, 16, b, 16, p, f, 31, None, None, None))
    # adjacent but disjoint is fine up to the modulus check
    assert L.poly_mul_modp(a, 16, b, 16, 4, a + 4 * 16, 31, r(n1), None) == pm.PM_EMODULUS
    q, rr = 0x300000, 0x400000
    assert rejected(L.poly_divrem_modp(a, 16, b, 8, p, a, 9, r(n1), rr, 8, r(n2), None))
    assert rejected(L.poly_divrem_modp(a, 16, b, 8, p, q, 9, r(n1), b + 4, 8, r(n2), None))
    assert rejected(L.poly_divrem_modp(a, 16, b, 8, p, q, 9, r(n1), q + 4 * 8, 8, r(n2), None))  # q and r
    assert rejected(L.poly_divrem_modp_naive(a, 16, b, 8, p, q, 9, r(n1), a, 8, r(n2), None))
    assert rejected(L.poly_divrem_modp_async(a, 16, b, 8, p, q, 9, None, b, 8, None, None, None))
    assert rejected(L.poly_gcd_modp(a, 16, b, 16, p, b + 4 * 15, 16, r(n1), None))
    assert rejected(L.poly_gcd_modp_naive(a, 16, b, 16, p, a, 16, r(n1), None))
    assert rejected(L.poly_gcd_modp_async(a, 16, b, 16, p, a, 16, None, None, None))
    degs = (ctypes.c_int64 * 40)()
    assert rejected(L.poly_gcd_modp_degrees(a, 16, b, 16, p, b, 16, r(n1), degs, 40, r(n2), None))
    assert rejected(L.poly_euclid_steps_modp(a, 16, b, 16, p, 3, q, 16, r(n1), q + 4 * 4, 16, r(n2), r(n3),
                                             None))
    g, s_, t = 0x500000, 0x600000, 0x700000
    assert rejected(L.poly_xgcd_modp(a, 16, b, 16, p, g, 16, r(n1), s_, 16, r(n2), g + 4 * 15, 16, r(n3), None))
    assert rejected(L.poly_xgcd_modp(a, 16, b, 16, p, g, 16, r(n1), a, 16, r(n2), t, 16, r(n3), None))
    assert n1.value == n2.value == n3.value == -7
    # batch items
    items = (pm.MulItem * 2)(pm.MulItem(a, 16, b, 16, p, 0x800000, 31), pm.MulItem(a, 16, b, 16, p, a, 31))
    batch = ctypes.c_void_p()
    assert rejected(L.pm_mul_batch_create(items, 2, 0, 0, ctypes.byref(batch)))
    gitems = (pm.GcdItem * 1)(pm.GcdItem(a, 16, b, 16, p, b, 16))
    assert rejected(L.pm_gcd_batch_create(gitems, 1, 0, ctypes.byref(batch)))
    assert not batch.value


def test_async_division_host_checks(L):
    """The asynchronous division plans from the given lengths: q_cap below
    na - nb + 1 or r_cap below min(na, nb - 1) is refused on the host, and
    b = 0 is PM_EDIVZERO."""
    a, b, q, r = 0x100000, 0x200000, 0x300000, 0x400000
    p = 469762049
    assert L.poly_divrem_modp_async(a, 16, b, 8, p, q, 8, None, r, 7, None, None, None) == pm.PM_EINVAL
    assert "q_cap" in pm.last_error()
    assert L.poly_divrem_modp_async(a, 16, b, 8, p, q, 9, None, r, 6, None, None, None) == pm.PM_EINVAL
    assert "r_cap" in pm.last_error()
    assert L.poly_divrem_modp_async(a, 5, b, 8, p, q, 0, None, r, 4, None, None, None) == pm.PM_EINVAL
    assert L.poly_divrem_modp_async(a, 16, b, 0, p, q, 9, None, r, 7, None, None, None) == pm.PM_EDIVZERO
    assert L.poly_divrem_modp_async(a, 16, b, 8, 9, q, 9, None, r, 7, None, None, None) == pm.PM_EMODULUS


def test_matrix_core_planner_keeps_digit_sums_exact():
    """Up to 2^26 terms per operand, square and lopsided, every product the
    planner gives the matrix cores has shares of at most 64 groups of 8
    block offsets (the bound on the int32 digit sums); the largest go to
    the VALU tiles instead. Host-only: the planner reads no device memory."""
    pm.set_params()
    sizes = [1 << k for k in range(8, 27)] + [3 * (1 << k) + 1 for k in range(8, 25)]
    seen = set()
    for na in sizes:
        for nb in (na, max(256, na // 64), 300, na // 2 + 17):
            info = pm.mul_plan(na, nb)
            seen.add(info["engine"])
            if info["engine"] == pm.MUL_MFMA:
                assert 1 <= info["max_share_groups"] <= 64, (na, nb, info)
                assert info["work_groups"] >= 1 and info["scratch_words"] > 0
            else:
                assert info["engine"] == pm.MUL_VALU and info["r"] in (1, 2, 4, 8, 16, 32), (na, nb, info)
    assert seen == {pm.MUL_VALU, pm.MUL_MFMA}
    assert pm.mul_plan(1 << 26, 1 << 26)["engine"] == pm.MUL_VALU  # beyond the exact matrix-core plans
    assert pm.mul_plan(65536, 65536)["engine"] == pm.MUL_MFMA
    assert pm.mul_plan(0, 5)["engine"] == 0
    # forcing the matrix cores does not override the bound
    pm.set_params(mul_engine=pm.MUL_MFMA)
    try:
        assert pm.mul_plan(1 << 26, 1 << 26)["engine"] == pm.MUL_VALU
        assert pm.mul_plan(3000, 3000)["engine"] == pm.MUL_MFMA
    finally:
        pm.set_params()


def test_workspace_sizes():
    pm.set_params()
    w_mul = pm.workspace_size(pm.PM_OP_MUL, 65536, 65536)
    assert w_mul == 64 + pm.mul_plan(65536, 65536)["scratch_words"]
    assert pm.workspace_size(pm.PM_OP_MUL, 0, 100) == 64
    assert pm.workspace_size(pm.PM_OP_DIVREM, 65536, 32768) >= 64 + 3 * 65536
    assert pm.workspace_size(pm.PM_OP_GCD, 32769, 32768) >= 64 + 4 * 32769
    with pytest.raises(pm.PolyModPError):
        pm.workspace_size(7, 10, 10)
    with pytest.raises(pm.PolyModPError):
        pm.workspace_size(pm.PM_OP_MUL, -1, 10)


def test_autotune_load(tmp_path):
    from paper_1402_0264_amd import tune
    pm.set_params()
    path = str(tmp_path / "params.txt")
    tune.save_params(path, {"mul_engine": pm.MUL_VALU, "mul_r": 8, "mul_s": 1024, "gcd_s": 64})
    pm.autotune_load(path)
    assert pm.get_params() == {"mul_s": 1024, "mul_r": 8, "div_s": 0, "gcd_s": 64, "mul_engine": 1}
    # a partial file keeps the other values; spacing, '=' and comments
    with open(path, "w") as fh:
        fh.write("# tuned\n\n  div_s = 16   # steps per chunk\n")
    pm.autotune_load(path)
    assert pm.get_params() == {"mul_s": 1024, "mul_r": 8, "div_s": 16, "gcd_s": 64, "mul_engine": 1}
    # any error leaves every value as it was
    for text in ("mul_r 3\n", "mul_s 512\nwarp 32\n", "gcd_s\n", "gcd_s 99999999999\n"):
        with open(path, "w") as fh:
            fh.write(text)
        with pytest.raises(pm.PolyModPError) as e:
            pm.autotune_load(path)
        assert e.value.status == pm.PM_EINVAL
        assert pm.get_params() == {"mul_s": 1024, "mul_r": 8, "div_s": 16, "gcd_s": 64, "mul_engine": 1}
    with pytest.raises(pm.PolyModPError):
        pm.autotune_load(str(tmp_path / "missing.txt"))
    pm.set_params()


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
