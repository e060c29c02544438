"""The product that allocates nothing (poly_mul_modp_noalloc, scratch in
a static device array) against the pooled asynchronous product
(poly_mul_modp_async) and the oracle, element by element, on two calls in
a row with the second one smaller, so that the second reuses the array the
first left holding its own partial sums."""
import numpy as np
import pytest

import oracle
import paper_1402_0264_amd as pm
from paper_1402_0264_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    pm.lib()
    pm.set_params()
    yield
    pm.set_params()


def _pair(st, na, nb, p):
    return st.uniform_poly(na - 1, p), st.uniform_poly(nb - 1, p)


def test_noalloc_equals_async_on_two_calls():
    import torch
    st = gen.Stream(gen.SEED_BASE + 301)
    p = gen.P_A
    # 20000 x 9000: the matrix cores (scratch = the shares' partial sums);
    # 3001 x 2500: the VALU tiles with 20 b-chunks (scratch = the rows of M)
    for na, nb in [(20000, 9000), (3001, 2500)]:
        a, b = _pair(st, na, nb, p)
        da, db = pm.to_device(a), pm.to_device(b)
        n = na + nb - 1
        f_pool = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        f_static = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        d_nf = torch.zeros(2, dtype=torch.int64, device="cuda")
        d_st = torch.full((2,), 7, dtype=torch.int32, device="cuda")
        pm.mul_async(da, db, p, f_pool, d_nf[0:1], d_st[0:1])
        pm.mul_noalloc(da, db, p, f_static, d_nf[1:2], d_st[1:2])
        torch.cuda.synchronize()
        assert d_st.tolist() == [0, 0], (na, nb)
        assert d_nf.tolist() == [n, n], (na, nb)
        got = pm.to_numpy(f_static)
        assert np.array_equal(got, pm.to_numpy(f_pool)), (na, nb)
        assert np.array_equal(got, oracle.mul(a, b, p)), (na, nb)


def test_noalloc_without_status_pointers_and_range_flag():
    import torch
    st = gen.Stream(gen.SEED_BASE + 302)
    p = gen.P_B
    a, b = _pair(st, 700, 650, p)
    f = torch.empty(700 + 650 - 1, dtype=torch.int32, device="cuda")
    pm.mul_noalloc(pm.to_device(a), pm.to_device(b), p, f)
    torch.cuda.synchronize()
    assert np.array_equal(pm.to_numpy(f), oracle.mul(a, b, p))
    bad = a.copy()
    bad[5] = p  # not a canonical residue
    d_nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    d_st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pm.mul_noalloc(pm.to_device(bad), pm.to_device(b), p, f, d_nf, d_st)
    torch.cuda.synchronize()
    assert int(d_st.item()) == pm.PM_ERANGE


def test_noalloc_rejects_a_plan_beyond_the_static_array():
    import torch
    # the VALU tiles with 64-coefficient b-chunks: 625 rows of 40063 words,
    # above the 2^24 words of the array; nothing is enqueued
    pm.set_params(mul_engine=pm.MUL_VALU, mul_s=64, mul_r=4)
    st = gen.Stream(gen.SEED_BASE + 303)
    a, b = _pair(st, 40000, 40000, gen.P_A)
    f = torch.full((79999,), -1, dtype=torch.int32, device="cuda")
    with pytest.raises(pm.PolyModPError) as e:
        pm.mul_noalloc(pm.to_device(a), pm.to_device(b), gen.P_A, f)
    assert e.value.status == pm.PM_EINVAL
    assert "static" in str(e.value)
    torch.cuda.synchronize()
    assert int((f != -1).sum().item()) == 0
