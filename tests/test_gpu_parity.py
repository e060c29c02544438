"""Bit-exact parity of the HIP library (through its C ABI) with the CPU
oracle, on seeded inputs: ragged sizes spanning several tiles, every prime
of the workloads plus tiny primes, the full-size workloads (sampled outputs
or size-independent properties where the oracle would be too slow), the
degenerate cases, and invariance under the tuning parameter s."""
import numpy as np
import pytest

import oracle
import paper_1402_0264_amd as pm
from paper_1402_0264_amd import gen
from tests import checkers as ck

pytestmark = pytest.mark.gpu

PRIMES = [gen.P_A, gen.P_B, gen.P_C]
TINY_ODD = [3, 5, 7, 65521]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    pm.lib()
    pm.set_params()
    yield
    pm.set_params()


def dev(x):
    return pm.to_device(x)


def host(t):
    return pm.to_numpy(t)


def rnd(st, n, p):
    return st.uniform_poly(n - 1, p) if n > 0 else np.zeros(0, dtype=np.uint32)


def same(x, y):
    return np.array_equal(np.asarray(x, dtype=np.uint32), np.asarray(y, dtype=np.uint32))


# ----------------------------------------------------------------- product
MUL_SIZES = [(1, 1), (1, 7), (7, 1), (2, 2), (63, 65), (100, 3), (257, 1000), (2048, 2048), (5000, 123),
             (4099, 4097), (12289, 700)]


@pytest.mark.parametrize("p", PRIMES + TINY_ODD + [2])
def test_mul_matches_oracle(p):
    st = gen.Stream(101 + p % 997)
    for na, nb in MUL_SIZES:
        a, b = rnd(st, na, p), rnd(st, nb, p)
        f = host(pm.mul(dev(a), dev(b), p))
        assert same(f, oracle.mul(a, b, p)), (p, na, nb)


ENGINE_SIZES = MUL_SIZES + [(64, 64), (65, 63), (2047, 2049), (2049, 2047), (4096, 64), (6000, 6000),
                             (33000, 257), (20000, 9000)]


@pytest.mark.parametrize("engine", [pm.MUL_VALU, pm.MUL_MFMA])
@pytest.mark.parametrize("p", PRIMES + [3, 65521, 2])
def test_mul_engines_match_oracle(engine, p):
    """Both product engines, forced, on ragged sizes (empty tails of every
    64-block, one or many output ranges of 2048, shares spanning ranges)."""
    st = gen.Stream(111 + p % 991)
    pm.set_params(mul_engine=engine)
    try:
        for na, nb in ENGINE_SIZES:
            a, b = rnd(st, na, p), rnd(st, nb, p)
            f = host(pm.mul(dev(a), dev(b), p))
            assert same(f, oracle.mul(a, b, p)), (engine, p, na, nb)
    finally:
        pm.set_params()


@pytest.mark.parametrize("p,n", [(gen.P_A, 65536), (gen.P_B, 65536), (gen.P_C, 65536), (gen.P_B, 262144)])
def test_mul_mfma_extreme_digits_full_size(p, n):
    """Every coefficient p - 1 (largest residues, so the largest digit sums
    the accumulators see; at 262144 the work-group shares reach their cap of
    512 block offsets): since (p-1)^2 = 1 mod p, f_k is the number of index
    pairs, min(k+1, n, 2n-1-k), mod p."""
    a = np.full(n, p - 1, dtype=np.uint32)
    pm.set_params(mul_engine=pm.MUL_MFMA)
    try:
        f = host(pm.mul(dev(a), dev(a), p)).astype(np.int64)
    finally:
        pm.set_params()
    k = np.arange(2 * n - 1, dtype=np.int64)
    want = np.minimum(np.minimum(k + 1, n), 2 * n - 1 - k) % p
    assert np.array_equal(f, want)


def test_mul_engines_identical_on_product_65536():
    a, b = gen.product_65536()
    p = gen.P_A
    da, db = dev(a), dev(b)
    out = {}
    for engine in (pm.MUL_VALU, pm.MUL_MFMA):
        pm.set_params(mul_engine=engine)
        try:
            out[engine] = host(pm.mul(da, db, p))
        finally:
            pm.set_params()
    assert same(out[pm.MUL_VALU], out[pm.MUL_MFMA])


def test_mul_mfma_range_error_and_async_status():
    import torch
    p = gen.P_A
    st = gen.Stream(112)
    a, b = rnd(st, 5000, p), rnd(st, 3000, p)
    pm.set_params(mul_engine=pm.MUL_MFMA)
    try:
        bad = b.copy(); bad[2999] = p + 5
        with pytest.raises(pm.PolyModPError) as e:
            pm.mul(dev(a), dev(bad), p)
        assert e.value.status == pm.PM_ERANGE
        bad = a.copy(); bad[0] = 0xFFFFFFFF
        with pytest.raises(pm.PolyModPError) as e:
            pm.mul(dev(bad), dev(b), p)
        assert e.value.status == pm.PM_ERANGE
        a_hz = np.concatenate([a, np.zeros(100, dtype=np.uint32)])
        f = torch.zeros(a_hz.size + b.size - 1, dtype=torch.int32, device="cuda")
        d_nf = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        d_st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        pm.mul_async(dev(a_hz), dev(b), p, f, d_nf, d_st)
        torch.cuda.synchronize()
        assert int(d_st.item()) == 0 and int(d_nf.item()) == a.size + b.size - 1
        assert same(host(f)[: a.size + b.size - 1], oracle.mul(a, b, p))
    finally:
        pm.set_params()


@pytest.mark.parametrize("r,s", [(1, 1), (2, 2), (4, 4), (8, 8), (16, 16), (4, 2048), (16, 512), (32, 64),
                                 (32, 4096), (1, 3), (8, 100)])
def test_mul_invariant_under_s(r, s):
    p = gen.P_B  # smallest fold interval
    st = gen.Stream(102)
    a, b = rnd(st, 3001, p), rnd(st, 2500, p)
    want = oracle.mul(a, b, p)
    pm.set_params(mul_r=r, mul_s=s)
    try:
        f = host(pm.mul(dev(a), dev(b), p))
    finally:
        pm.set_params()
    assert same(f, want)


def test_mul_product_2048():
    a, b = gen.product_2048()
    f = host(pm.mul(dev(a), dev(b), gen.P_A))
    assert f.size == 4095
    assert same(f, oracle.mul(a, b, gen.P_A))


def test_mul_product_65536_full():
    """Full size, every output coefficient against the oracle's product,
    plus the evaluation identity at random points."""
    a, b = gen.product_65536()
    p = gen.P_A
    f = host(pm.mul(dev(a), dev(b), p))
    assert f.size == 131071
    assert same(f, oracle.mul(a, b, p))
    st = gen.Stream(103)
    for _ in range(3):
        x = st.uniform_int(0, p - 1)
        assert ck.horner(f, x, p) == ck.horner(a, x, p) * ck.horner(b, x, p) % p


def test_mul_edge_cases():
    p = gen.P_A
    z = np.zeros(0, dtype=np.uint32)
    st = gen.Stream(104)
    a = rnd(st, 40, p)
    assert pm.mul(dev(a), dev(z), p).numel() == 0
    assert pm.mul(dev(z), dev(a), p).numel() == 0
    a_hz = np.concatenate([a, np.zeros(13, dtype=np.uint32)])   # high zeros are ignored
    b = rnd(st, 17, p)
    b_hz = np.concatenate([b, np.zeros(300, dtype=np.uint32)])
    f = host(pm.mul(dev(a_hz), dev(b_hz), p))
    assert same(f, oracle.mul(a, b, p))
    assert same(host(pm.mul(dev(np.zeros(5, dtype=np.uint32)), dev(b), p)), [])
    bad = a.copy(); bad[3] = p
    with pytest.raises(pm.PolyModPError) as e:
        pm.mul(dev(bad), dev(b), p)
    assert e.value.status == pm.PM_ERANGE


def test_mul_async_writes_device_results():
    import torch
    p = gen.P_C
    st = gen.Stream(105)
    a, b = rnd(st, 1500, p), rnd(st, 900, p)
    f = torch.zeros(2399, dtype=torch.int32, device="cuda")
    d_nf = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    d_st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    pm.mul_async(dev(a), dev(b), p, f, d_nf, d_st)
    torch.cuda.synchronize()
    assert int(d_nf.item()) == 2399 and int(d_st.item()) == 0
    assert same(host(f), oracle.mul(a, b, p))


# ---------------------------------------------------------------- division
DIV_SIZES = [(1, 1), (10, 1), (10, 3), (100, 99), (500, 17), (300, 300), (3, 10), (2049, 2048), (5000, 200),
             (20000, 64), (1000, 999), (700, 2)]


@pytest.mark.parametrize("p", PRIMES + TINY_ODD + [2])
def test_divrem_matches_oracle(p):
    st = gen.Stream(201 + p % 997)
    for na, nb in DIV_SIZES:
        a, b = rnd(st, na, p), rnd(st, nb, p)
        q, r = pm.divrem(dev(a), dev(b), p)
        wq, wr = oracle.divrem(a, b, p)
        assert same(host(q), wq) and same(host(r), wr), (p, na, nb)


@pytest.mark.parametrize("s", [1, 2, 5, 16, 64])
def test_divrem_invariant_under_s(s):
    p = gen.P_A
    st = gen.Stream(202)
    a, b = rnd(st, 3000, p), rnd(st, 1100, p)
    wq, wr = oracle.divrem(a, b, p)
    pm.set_params(div_s=s)
    try:
        q, r = pm.divrem(dev(a), dev(b), p)
    finally:
        pm.set_params()
    assert same(host(q), wq) and same(host(r), wr)


# Long quotients run on many cooperating blocks (runs of about 512 head
# positions each); divisors from degree 1 up, every s kind (1, odd, 64).
LONG_DIV = [(40000, 3000, 1), (40000, 3000, 3), (40000, 3000, 17), (40000, 3000, 64), (50000, 2, 64),
            (50000, 40, 7), (20000, 19000, 64), (70000, 600, 64), (9000, 70, 64)]


@pytest.mark.parametrize("na,nb,s", LONG_DIV)
def test_divrem_long_quotient(na, nb, s):
    p = gen.P_B
    st = gen.Stream(204 + na % 1000 + nb + s)
    a, b = rnd(st, na, p), rnd(st, nb, p)
    wq, wr = oracle.divrem(a, b, p)
    pm.set_params(div_s=s)
    try:
        q, r = pm.divrem(dev(a), dev(b), p)
    finally:
        pm.set_params()
    assert same(host(q), wq) and same(host(r), wr), (na, nb, s)


@pytest.mark.parametrize("p", [2, 3, gen.P_C])
def test_divrem_long_quotient_small_and_other_primes(p):
    st = gen.Stream(207 + p % 1000)
    for na, nb, s in [(30000, 700, 64), (12000, 5, 9), (9000, 8900, 1)]:
        a, b = rnd(st, na, p), rnd(st, nb, p)
        wq, wr = oracle.divrem(a, b, p)
        pm.set_params(div_s=s)
        try:
            q, r = pm.divrem(dev(a), dev(b), p)
        finally:
            pm.set_params()
        assert same(host(q), wq) and same(host(r), wr), (p, na, nb, s)


def test_divrem_head_longer_than_planned():
    # zeros above the top coefficient of b: the head is longer than the
    # lengths suggest, so blocks own several runs of it
    p = gen.P_A
    st = gen.Stream(205)
    a = rnd(st, 30000, p)
    b = np.concatenate([rnd(st, 1000, p), np.zeros(20000, dtype=np.uint32)])
    q, r = pm.divrem(dev(a), dev(b), p)
    wq, wr = oracle.divrem(a, b, p)
    assert host(q).size == 29001
    assert same(host(q), wq) and same(host(r), wr)


def test_divrem_full_size_65536_by_32768():
    # the division workload of the s sweep: 32769 quotient terms
    p = gen.P_A
    st = gen.Stream(206)
    a, b = rnd(st, 65536, p), rnd(st, 32768, p)
    q, r = pm.divrem(dev(a), dev(b), p)
    wq, wr = oracle.divrem(a, b, p)
    assert same(host(q), wq) and same(host(r), wr)


def test_divrem_gcd_workload():
    pl = gen.gcd_32768()
    p = pl.p
    a = oracle.mul(pl.g, pl.u, p)
    b = oracle.mul(pl.g, pl.v, p)
    q, r = pm.divrem(dev(a), dev(b), p)
    wq, wr = oracle.divrem(a, b, p)
    assert host(q).size == 2
    assert same(host(q), wq) and same(host(r), wr)


def test_divrem_edge_cases():
    p = gen.P_B
    st = gen.Stream(203)
    a, b = rnd(st, 50, p), rnd(st, 9, p)
    z = np.zeros(4, dtype=np.uint32)
    with pytest.raises(pm.PolyModPError) as e:
        pm.divrem(dev(a), dev(z), p)
    assert e.value.status == pm.PM_EDIVZERO
    for x, y in [(a, b), (b, a), (np.zeros(0, dtype=np.uint32), b), (a, a), (a, np.array([7], dtype=np.uint32)),
                 (np.concatenate([a, np.zeros(5, dtype=np.uint32)]), np.concatenate([b, np.zeros(50, dtype=np.uint32)]))]:
        q, r = pm.divrem(dev(x), dev(y), p)
        wq, wr = oracle.divrem(x, y, p)
        assert same(host(q), wq) and same(host(r), wr)
    bad = b.copy(); bad[0] = p + 5
    with pytest.raises(pm.PolyModPError) as e:
        pm.divrem(dev(a), dev(bad), p)
    assert e.value.status == pm.PM_ERANGE


# The naive division (one step per launch), the s = 1 end of the sweep.
@pytest.mark.parametrize("p", [gen.P_A, gen.P_B, 3, 2])
def test_divrem_naive_matches_oracle(p):
    st = gen.Stream(208 + p % 997)
    for na, nb in [(1, 1), (10, 1), (10, 3), (100, 99), (500, 17), (300, 300), (3, 10), (2049, 2048), (3000, 1100),
                   (1000, 999), (700, 2)]:
        a, b = rnd(st, na, p), rnd(st, nb, p)
        q, r = pm.divrem(dev(a), dev(b), p, naive=True)
        wq, wr = oracle.divrem(a, b, p)
        assert same(host(q), wq) and same(host(r), wr), (p, na, nb)


def test_divrem_naive_edge_cases():
    p = gen.P_B
    st = gen.Stream(209)
    a, b = rnd(st, 50, p), rnd(st, 9, p)
    with pytest.raises(pm.PolyModPError) as e:
        pm.divrem(dev(a), dev(np.zeros(4, dtype=np.uint32)), p, naive=True)
    assert e.value.status == pm.PM_EDIVZERO
    for x, y in [(np.zeros(0, dtype=np.uint32), b), (a, a), (a, np.array([7], dtype=np.uint32)),
                 (np.concatenate([a, np.zeros(5, dtype=np.uint32)]), np.concatenate([b, np.zeros(50, dtype=np.uint32)]))]:
        q, r = pm.divrem(dev(x), dev(y), p, naive=True)
        wq, wr = oracle.divrem(x, y, p)
        assert same(host(q), wq) and same(host(r), wr)
    bad = b.copy(); bad[0] = p + 5
    with pytest.raises(pm.PolyModPError) as e:
        pm.divrem(dev(a), dev(bad), p, naive=True)
    assert e.value.status == pm.PM_ERANGE


# --------------------------------------------------------------------- gcd
GCD_CASES = [(5, 3, 0), (40, 40, 3), (100, 60, 20), (60, 100, 59), (200, 199, 50), (300, 300, 0),
             (1000, 999, 10), (2500, 2400, 700), (5000, 4999, 1234), (3000, 10, 2), (700, 1, 0)]


@pytest.mark.parametrize("p", PRIMES + TINY_ODD)
def test_gcd_matches_oracle(p):
    st = gen.Stream(301 + p % 997)
    for da, db, dg in GCD_CASES:
        pl = gen.planted_gcd(da, db, dg, p, st)
        a, b = oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)
        g = host(pm.gcd(dev(a), dev(b), p))
        assert same(g, oracle.gcd(a, b, p)), (p, da, db, dg)


@pytest.mark.parametrize("s", [1, 2, 7, 31, 64, 128, 256])
def test_gcd_invariant_under_s(s):
    p = gen.P_C
    st = gen.Stream(302)
    pl = gen.planted_gcd(3000, 2999, 300, p, st)
    a, b = oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)
    want = oracle.gcd(a, b, p)
    pm.set_params(gcd_s=s)
    try:
        g = host(pm.gcd(dev(a), dev(b), p))
    finally:
        pm.set_params()
    assert same(g, want)


def test_gcd_workload_32768():
    pl = gen.gcd_32768()
    p = pl.p
    a = oracle.mul(pl.g, pl.u, p)
    b = oracle.mul(pl.g, pl.v, p)
    g = host(pm.gcd(dev(a), dev(b), p))
    want, degs, stats = oracle.gcd(a, b, p, with_info=True)
    assert same(g, want) and same(g, pl.g)
    got = pm.last_gcd_stats()
    assert got["steps"] == stats.steps and got["updates"] == stats.updates


# The naive gcd (one division step per launch, exact inverses): the monic
# gcd and the exact step and update counts of the oracle.
@pytest.mark.parametrize("p", [gen.P_A, gen.P_C, 3, 2])
def test_gcd_naive_matches_oracle(p):
    st = gen.Stream(304 + p % 997)
    for da, db, dg in [(5, 3, 0), (40, 40, 3), (100, 60, 20), (60, 100, 59), (200, 199, 50), (300, 300, 0),
                       (1000, 999, 10), (2500, 2400, 700)]:
        pl = gen.planted_gcd(da, db, dg, p, st)
        a, b = oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)
        g = host(pm.gcd(dev(a), dev(b), p, naive=True))
        want, degs, stats = oracle.gcd(a, b, p, with_info=True)
        assert same(g, want), (p, da, db, dg)
        got = pm.last_gcd_stats()
        assert got["steps"] == stats.steps and got["updates"] == stats.updates, (p, da, db, dg)
    z = np.zeros(0, dtype=np.uint32)
    x = rnd(st, 30, p)
    for u, v in [(z, z), (x, z), (z, x), (x, x), (x, np.array([1], dtype=np.uint32))]:
        assert same(host(pm.gcd(dev(u), dev(v), p, naive=True)), oracle.gcd(u, v, p))


@pytest.mark.parametrize("p", [3, 5, gen.P_A])
def test_gcd_counts_match_oracle(p):
    # steps and updates as the oracle counts them, also when leading
    # coefficients vanish (small primes): one block and the cooperative grid
    st = gen.Stream(305 + p % 997)
    for da, db, dg in [(40, 40, 3), (200, 199, 50), (1000, 999, 10), (6000, 5999, 100)]:
        pl = gen.planted_gcd(da, db, dg, p, st)
        a, b = oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)
        g = host(pm.gcd(dev(a), dev(b), p))
        want, degs, stats = oracle.gcd(a, b, p, with_info=True)
        assert same(g, want), (p, da, db, dg)
        got = pm.last_gcd_stats()
        assert got["steps"] == stats.steps and got["updates"] == stats.updates, (p, da, db, dg, got, stats.steps)


@pytest.mark.parametrize("p", [3, gen.P_A])
def test_gcd_leading_division(p):
    # a degree gap of 128 or more starts with one Euclidean division; the
    # gcd and the step and update counts stay the oracle's in both
    # orientations (b of higher degree stops one position early, Sec. 6's
    # tie rule), on one block and on the cooperative grid
    st = gen.Stream(306 + p % 997)
    cases = []
    for da, db, dg in [(1000, 300, 10), (300, 1000, 10), (500, 372, 5), (372, 500, 5), (500, 373, 5),
                       (6000, 2000, 50), (2000, 6000, 50), (3000, 40, 0)]:
        pl = gen.planted_gcd(da, db, dg, p, st)
        cases.append((oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p), (da, db, dg)))
    # b = a x q' + r: the division's constant quotient term is zero
    a = st.uniform_poly(400, p)
    b = oracle.mul(a, np.concatenate([np.zeros(1, np.uint32), st.uniform_poly(300, p)]), p)
    r = st.uniform_poly(250, p)
    b[:r.size] = (b[:r.size].astype(np.uint64) + r) % p
    cases.append((a, b.astype(np.uint32), "q0 = 0"))
    # constant divisors, b_0 = 0 and b_0 != 0
    c = np.array([2], dtype=np.uint32)
    x = st.uniform_poly(300, p)
    x0 = x.copy(); x0[0] = 0
    cases += [(x, c, "const b"), (c, x, "const a"), (c, x0, "const a, b_0 = 0")]
    # leading zeros: the term counts differ by more than the true degrees
    pl = gen.planted_gcd(200, 199, 7, p, st)
    pad = np.concatenate([oracle.mul(pl.g, pl.u, p), np.zeros(200, dtype=np.uint32)])
    cases.append((pad, oracle.mul(pl.g, pl.v, p), "padded"))
    for u, v, tag in cases:
        g = host(pm.gcd(dev(u), dev(v), p))
        want, degs, stats = oracle.gcd(u, v, p, with_info=True)
        assert same(g, want), (p, tag)
        got = pm.last_gcd_stats()
        assert got["steps"] == stats.steps and got["updates"] == stats.updates, (p, tag, got, stats.steps)


@pytest.mark.parametrize("p", [3, 5, gen.P_A])
def test_xgcd_matches_oracle(p):
    # (g, s, t) bit-exact against the oracle's extended Euclid: planted pairs
    # in both orientations, leading degree gaps (both orientations, q_0 = 0),
    # one block and the cooperative grid, and the degenerate inputs
    st = gen.Stream(307 + p % 997)
    cases = []
    for da, db, dg in [(5, 3, 0), (3, 5, 0), (40, 40, 3), (200, 199, 50), (199, 200, 50), (1000, 999, 10),
                       (1000, 300, 10), (300, 1000, 10), (3000, 40, 0), (6000, 5999, 100), (2000, 6000, 50)]:
        pl = gen.planted_gcd(da, db, dg, p, st)
        cases.append((oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p), (da, db, dg)))
    a = st.uniform_poly(400, p)
    b = oracle.mul(a, np.concatenate([np.zeros(1, np.uint32), st.uniform_poly(300, p)]), p)
    r = st.uniform_poly(250, p)
    b[:r.size] = (b[:r.size].astype(np.uint64) + r) % p
    cases.append((a, b.astype(np.uint32), "q0 = 0"))
    x = st.uniform_poly(60, p)
    xy = oracle.mul(x, st.uniform_poly(20, p), p)
    xbig = oracle.mul(x, st.uniform_poly(300, p), p)
    c = np.array([2], dtype=np.uint32)
    z = np.zeros(0, dtype=np.uint32)
    pad = np.concatenate([x, np.zeros(7, dtype=np.uint32)])
    cases += [(x, x, "a = b"), (x, xy, "a | b"), (xy, x, "b | a"), (xbig, x, "b | a, gap"), (x, xbig, "a | b, gap"),
              (x, z, "b = 0"), (z, x, "a = 0"), (z, z, "both 0"), (c, x, "const a"), (x, c, "const b"),
              (pad, xy, "padded")]
    for u, v, tag in cases:
        g, s_, t_ = (host(y) for y in pm.xgcd(dev(u), dev(v), p))
        wg, ws, wt = oracle.xgcd(u, v, p)
        assert same(g, wg) and same(s_, ws) and same(t_, wt), (p, tag)
        if g.size:
            want, degs, stats = oracle.gcd(u, v, p, with_info=True)
            got = pm.last_gcd_stats()
            assert got["steps"] == stats.steps and got["updates"] == stats.updates, (p, tag)


def test_xgcd_workload_32768_certificate():
    # the degree 32768 / 32767 pair with a planted degree-1000 gcd: g is the
    # planted one and s a + t b = g, checked by the product path against the
    # oracle's product at sampled coefficients and in full on the device
    pl = gen.gcd_32768()
    p = pl.p
    gd = pm.to_device(pl.g)
    a = pm.mul(gd, pm.to_device(pl.u), p)
    b = pm.mul(gd, pm.to_device(pl.v), p)
    g, s_, t_ = pm.xgcd(a, b, p)
    assert same(host(g), pl.g)
    assert s_.numel() - 1 < (b.numel() - 1) - (g.numel() - 1)
    sa = pm.mul(s_, a, p)
    tb = pm.mul(t_, b, p)
    n = max(sa.numel(), tb.numel())
    lhs = np.zeros(n, dtype=np.uint64)
    lhs[:sa.numel()] += host(sa)
    lhs[:tb.numel()] += host(tb)
    lhs %= p
    want = np.zeros(n, dtype=np.uint64)
    want[:pl.g.size] = pl.g
    assert np.array_equal(lhs, want)
    hs, ha = host(s_), host(a)
    rng = np.random.default_rng(5)
    for k in rng.integers(0, sa.numel(), 8):
        assert oracle.mul_coeff(hs, ha, p, int(k)) == int(host(sa)[k])


def test_gcd_and_xgcd_grid_multi_pass_slices():
    # degree 300000: more than 2 x 256 slices of 512 positions, so the
    # cooperative grid takes slices of 1024 and each apply wave walks its
    # half-slice in two passes of 256 positions. The oracle's gcd is too
    # slow here: the planted monic g is the answer (u, v coprime with
    # probability about 1 - 1/p), and s a + t b = g is checked in full on the
    # device with sampled product coefficients against the oracle.
    p = gen.P_A
    pl = gen.planted_gcd(300000, 299999, 16, p, gen.Stream(gen.SEED_BASE + 61))
    gd = pm.to_device(pl.g)
    a = pm.mul(gd, pm.to_device(pl.u), p)
    b = pm.mul(gd, pm.to_device(pl.v), p)
    ha, hb = host(a), host(b)
    rng = np.random.default_rng(61)
    for k in rng.integers(0, ha.size, 4):
        assert oracle.mul_coeff(pl.g, pl.u, p, int(k)) == int(ha[k])
        assert oracle.mul_coeff(pl.g, pl.v, p, int(k)) == int(hb[k])
    assert same(host(pm.gcd(a, b, p)), pl.g)
    st = pm.last_gcd_stats()
    assert st["chunks"] > 0 and st["steps"] > 0
    g, s_, t_ = pm.xgcd(a, b, p)
    assert same(host(g), pl.g)
    assert s_.numel() - 1 < (b.numel() - 1) - (g.numel() - 1)
    sa = pm.mul(s_, a, p)
    tb = pm.mul(t_, b, p)
    n = max(sa.numel(), tb.numel())
    lhs = np.zeros(n, dtype=np.uint64)
    lhs[:sa.numel()] += host(sa)
    lhs[:tb.numel()] += host(tb)
    lhs %= p
    want = np.zeros(n, dtype=np.uint64)
    want[:pl.g.size] = pl.g
    assert np.array_equal(lhs, want)


@pytest.mark.parametrize("p", [3, gen.P_A])
def test_gcd_grid_big_steps_and_rescans(p):
    # the cooperative kernel at several blocks: degree gaps of 64-127 (no
    # leading division, so the first steps are single big steps through
    # the grid), and at p = 3 frequent vanishing leading coefficients
    # (chunks that end with an unknown degree and a rescan); the gcd, the
    # counts and the extended gcd's cofactors are the oracle's
    st = gen.Stream(308 + p % 997)
    for da, db, dg in [(6000, 5900, 40), (5900, 6000, 40), (3000, 2936, 7), (9000, 8999, 500)]:
        pl = gen.planted_gcd(da, db, dg, p, st)
        a, b = oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)
        g = host(pm.gcd(dev(a), dev(b), p))
        want, degs, stats = oracle.gcd(a, b, p, with_info=True)
        assert same(g, want), (p, da, db)
        got = pm.last_gcd_stats()
        assert got["steps"] == stats.steps and got["updates"] == stats.updates, (p, da, db)
        gx, sx, tx = (host(y) for y in pm.xgcd(dev(a), dev(b), p))
        wg, ws, wt = oracle.xgcd(a, b, p)
        assert same(gx, wg) and same(sx, ws) and same(tx, wt), (p, da, db, "xgcd")


def test_gcd_edge_cases():
    p = gen.P_A
    st = gen.Stream(303)
    a, b = rnd(st, 30, p), rnd(st, 12, p)
    z = np.zeros(0, dtype=np.uint32)
    cases = [(z, z), (a, z), (z, a), (a, a), (a, np.array([9], dtype=np.uint32)), (a, b),
             (np.concatenate([a, np.zeros(9, dtype=np.uint32)]), np.zeros(3, dtype=np.uint32))]
    h = rnd(st, 8, p)
    ab = oracle.mul(a, h, p)
    cases.append((ab, a))   # a | ab
    for x, y in cases:
        g = host(pm.gcd(dev(x), dev(y), p))
        assert same(g, oracle.gcd(x, y, p))
    for i, j in [(12, 18), (97, 13), (64, 48)]:   # gcd(X^i - 1, X^j - 1) = X^gcd(i,j) - 1
        x = np.zeros(i + 1, dtype=np.uint32); x[0] = p - 1; x[i] = 1
        y = np.zeros(j + 1, dtype=np.uint32); y[0] = p - 1; y[j] = 1
        assert same(host(pm.gcd(dev(x), dev(y), p)), oracle.gcd(x, y, p))
    bad = a.copy(); bad[-1] = p
    with pytest.raises(pm.PolyModPError) as e:
        pm.gcd(dev(bad), dev(b), p)
    assert e.value.status == pm.PM_ERANGE


def test_gcd_batch_mixed_primes_and_degrees():
    """One launch, one block per instance, both kernel shapes (<= 4096 and
    up to the batch limit), three primes; each result equals the oracle's
    and equals the result of the same instance computed alone."""
    st = gen.Stream(304)
    pairs, want = [], []
    for i in range(40):
        p = gen.PRIMES[st.index(3)]
        D = st.log_uniform_int(8, 3000) if i < 36 else st.log_uniform_int(4097, 9000)
        k = st.uniform_int(0, D // 4)
        pl = gen.planted_gcd(D, D - 1, k, p, st)
        a, b = oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)
        pairs.append((a, b, p))
        want.append(oracle.gcd(a, b, p))
    res = pm.gcd_batch([(dev(a), dev(b), p) for a, b, p in pairs])
    for (g, info), w in zip(res, want):
        assert info["status"] == 0
        assert same(host(g), w)
    a, b, p = pairs[5]
    assert same(host(pm.gcd(dev(a), dev(b), p)), want[5])


def test_gcd_batch_reports_item_errors():
    p = gen.P_A
    st = gen.Stream(305)
    a, b = rnd(st, 20, p), rnd(st, 10, p)
    bad = a.copy(); bad[0] = p + 1
    c, d = rnd(st, 15, gen.P_C), rnd(st, 7, gen.P_C)
    res = pm.gcd_batch([(dev(a), dev(b), p), (dev(bad), dev(b), p), (dev(c), dev(d), gen.P_C),
                        (dev(a), dev(b), gen.P_C)])
    assert res[0][1]["status"] == 0 and same(host(res[0][0]), oracle.gcd(a, b, p))
    assert res[1][1]["status"] == pm.PM_ERANGE
    assert res[2][1]["status"] == 0 and same(host(res[2][0]), oracle.gcd(c, d, gen.P_C))
    # residues of P_A are not all below P_C
    assert res[3][1]["status"] == (pm.PM_ERANGE if (a >= gen.P_C).any() or (b >= gen.P_C).any() else 0)


# ---------------------------------------------------------- batched product
def _batch_items(count, lo, hi, seed, primes=PRIMES):
    st = gen.Stream(seed)
    items = []
    for _ in range(count):
        p = primes[st.index(len(primes))]
        na, nb = st.log_uniform_int(lo, hi), st.log_uniform_int(lo, hi)
        items.append((st.uniform_poly(na - 1, p), st.uniform_poly(nb - 1, p), p))
    return items


@pytest.mark.parametrize("r,kc", [(0, 0), (4, 64), (8, 1000), (16, 2048), (4, 4)])
def test_mul_batch_matches_oracle(r, kc):
    items = _batch_items(150, 1, 3000, 401)
    b = pm.MulBatch([(dev(a), dev(b_), p) for a, b_, p in items], r, kc)
    b.run()
    import torch
    torch.cuda.synchronize()
    for (a, b_, p), f in zip(items, b.outputs):
        assert same(host(f), oracle.mul(a, b_, p))
    b.close()


def _edge_batch_items():
    """Ragged and degenerate shapes for the batch engines: single
    coefficients, lengths on and beside the 64-coefficient blocks and the
    4096-output ranges, one operand far longer than the other, the longest
    shorter operand the matrix cores take (32704) and one past it, and
    p = 2 and 3."""
    st = gen.Stream(gen.SEED_BASE + 407)
    shapes = [(1, 1), (1, 5), (7, 1), (63, 64), (64, 65), (65, 63), (4096, 1), (4095, 2), (4097, 64),
              (2049, 2048), (3000, 3001), (8192, 8192), (8193, 257), (20000, 300), (32704, 40),
              (40, 32704), (32705, 32705), (5000, 4100), (129, 127), (256, 256), (1000, 1024)]
    items = []
    for i, (na, nb) in enumerate(shapes):
        p = (2, 3, gen.P_A, 998244353)[i % 4]
        items.append((st.uniform_poly(na - 1, p), st.uniform_poly(nb - 1, p), p))
    # every coefficient 0x808080 (signed digits -128, -127, -127, 1) at the
    # longest b the matrix cores take: digit sums at the int32 bound
    w = np.full(32704, 0x808080, dtype=np.uint32)
    items.append((w, w.copy(), gen.P_A))
    return items


@pytest.mark.parametrize("engine", [pm.MUL_AUTO, pm.MUL_VALU, pm.MUL_MFMA])
def test_mul_batch_engines_match_oracle(engine):
    """The batch with every item on the VALU tiles, on the matrix cores
    where they apply, and split by the cost model: each output element
    against the oracle's product."""
    import torch
    items = _edge_batch_items() + _batch_items(80, 1, 9000, 408)
    pm.set_params(mul_engine=engine)
    try:
        b = pm.MulBatch([(dev(a), dev(b_), p) for a, b_, p in items])
    finally:
        pm.set_params()
    b.run()
    torch.cuda.synchronize()
    want = oracle_mul_many([(a, b_) for a, b_, _ in items], None, [p for _, _, p in items])
    for i, f in enumerate(b.outputs):
        assert same(host(f), want[i]), (engine, i, items[i][0].size, items[i][1].size)
    b.close()


def test_mul_batch_graph_replay_and_status():
    import torch
    items = _batch_items(60, 1, 2000, 402)
    bad_a = items[7][0].copy(); bad_a[0] = items[7][2]
    items[7] = (bad_a, items[7][1], items[7][2])
    b = pm.MulBatch([(dev(a), dev(b_), p) for a, b_, p in items], 8, 256)
    status = torch.full((len(items),), 77, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run(status, stream=s)          # once outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[7] == pm.PM_ERANGE and (np.delete(st, 7) == 0).all()
    want = [oracle.mul(a, b_, p) for a, b_, p in items]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        for f in b.outputs:
            f.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, f in enumerate(b.outputs):
            if i != 7:
                assert same(host(f), want[i]), (rep, i)
    b.close()


def test_mul_batch_two_engines_side_stream_in_a_graph():
    """r = 4 with items for both engines: the VALU tiles run on the batch's
    second stream beside the matrix cores, joined back by events. Captured
    in a graph and replayed three times (outputs cleared between, the
    program's own work and syncs between replays); every replay against the
    oracle element by element."""
    import torch
    items = _batch_items(40, 2000, 9000, 409) + _batch_items(120, 1, 400, 410)
    b = pm.MulBatch([(dev(a), dev(b_), p) for a, b_, p in items], 4, 512)
    want = oracle_mul_many([(a, b_) for a, b_, _ in items], None, [p for _, _, p in items])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for i, f in enumerate(b.outputs):
        assert same(host(f), want[i]), ("eager", i)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        for f in b.outputs:
            f.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, f in enumerate(b.outputs):
            assert same(host(f), want[i]), (rep, i)
    b.close()


def oracle_mul_many(pairs, p, primes=None):
    """The oracle's product of every pair (modulo p, or primes[i] for pair
    i), on a pool of host threads (the C oracle runs without the
    interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    ps = primes if primes is not None else [p] * len(pairs)
    with ThreadPoolExecutor(max_workers=min(16, max(1, len(pairs)))) as ex:
        return list(ex.map(lambda i: oracle.mul(pairs[i][0], pairs[i][1], ps[i]), range(len(pairs))))


def test_mul_batch_workload_4096_full():
    """The 4096-product workload: every output coefficient of every product
    against the oracle's product."""
    import torch
    bt = gen.batch_products()
    p = bt.p
    b = pm.MulBatch([(dev(a), dev(b_), p) for a, b_ in zip(bt.a, bt.b)])
    b.run()
    torch.cuda.synchronize()
    want = oracle_mul_many(list(zip(bt.a, bt.b)), p)
    for i, f in enumerate(b.outputs):
        assert same(host(f), want[i]), i
    b.close()


def test_mul_s1_plan_beyond_one_launch_of_blocks():
    """s = 1 on a 65536 x 8192 product: 8192 b-chunks x 256 tiles exceed
    2^20 thread-blocks, so the blocks stride over the work; sampled outputs
    against the oracle, and the same result as s = 512."""
    import torch
    p = gen.P_A
    a, b = gen.mul_pair(65536, 8192, p, seed=gen.SEED_BASE + 60)
    pm.set_params(mul_r=1, mul_s=1)
    try:
        f1 = pm.mul(dev(a), dev(b), p)
    finally:
        pm.set_params()
    torch.cuda.synchronize()
    fh = host(f1)
    st = gen.Stream(106)
    for k in [0, 1, 8190, 8191, 65535, 73726] + [st.uniform_int(0, 73726) for _ in range(20)]:
        assert int(fh[k]) == oracle.mul_coeff(a, b, p, k), k
    pm.set_params(mul_r=16, mul_s=512)
    try:
        f2 = pm.mul(dev(a), dev(b), p)
    finally:
        pm.set_params()
    assert torch.equal(f1, f2)
    pm.release()  # drop the 2 GiB partial-sum pool


# ------------------------------------------------------------------ server
def _served_requests(count, seed, lo=8, hi=6000):
    st = gen.Stream(seed)
    reqs = []
    for _ in range(count):
        p = gen.PRIMES[st.index(3)]
        D = st.log_uniform_int(lo, hi)
        k = st.uniform_int(0, D // 4)
        pl = gen.planted_gcd(D, D - 1, k, p, st)
        reqs.append((oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p), p))
    return reqs


def test_gcd_batch_graph_replay():
    # the prepared gcd batch: two block shapes, three primes, one bad item,
    # run eagerly and then replayed from a captured graph with eager work
    # in between; every replay gives the oracle's gcds and counts again
    import torch
    reqs = _served_requests(40, 506, lo=8, hi=6000)
    bad_a = reqs[5][0].copy()
    bad_a[0] = reqs[5][2]
    reqs[5] = (bad_a, reqs[5][1], reqs[5][2])
    want = [oracle.gcd(a, b, p, with_info=True) if i != 5 else None for i, (a, b, p) in enumerate(reqs)]
    batch = pm.GcdBatch([(dev(a), dev(b), p) for a, b, p in reqs], s=64)

    def check(tag):
        for i, (g, r) in enumerate(batch.results()):
            if i == 5:
                assert r["status"] == pm.PM_ERANGE, tag
                continue
            wg, degs, stats = want[i]
            assert r["status"] == 0 and same(host(g), wg), (tag, i)
            assert r["steps"] == stats.steps and r["updates"] == stats.updates, (tag, i)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.run(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    check("eager")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.run()
    x = torch.arange(1 << 16, device="cuda", dtype=torch.int64)
    for rep in range(3):
        for g in batch.gs:
            g.fill_(-1)
        y = (x * rep).sum()              # the program's own work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert int(y) == rep * ((1 << 16) * ((1 << 16) - 1) // 2)
        check("replay %d" % rep)
    batch.close()


def test_server_results_same_alone_and_in_the_mix():
    reqs = _served_requests(48, 501) + _served_requests(3, 502, lo=5000, hi=16000)
    want = [oracle.gcd(a, b, p) for a, b, p in reqs]
    srv = pm.Server()
    tickets = {}
    done = {}
    # submit in three waves while polling, so later requests join a GPU
    # that is already working on earlier ones
    for w in range(3):
        for i in range(w, len(reqs), 3):
            a, b, p = reqs[i]
            tickets[srv.submit(a, b, p, tag=i)] = i
        for c in srv.poll():
            done[c["tag"]] = c
    for c in srv.drain():
        done[c["tag"]] = c
    assert len(done) == len(reqs)
    for i, w in enumerate(want):
        assert done[i]["status"] == 0 and same(done[i]["g"], w), i
    srv.close()
    # alone: a fresh server, one request at a time
    for i in [0, 7, len(reqs) - 1]:
        solo = pm.Server()
        solo.submit(*reqs[i], tag=i)
        c = solo.drain()[0]
        assert same(c["g"], done[i]["g"]) and c["steps"] == done[i]["steps"]
        solo.close()


def test_server_batch_submission():
    # one call submits many requests: the first ones start while the rest are
    # copied, more than the slots hold wait in the queue, and the results
    # equal the oracle's; a batch with one bad request queues none of them
    reqs = _served_requests(40, 504, lo=8, hi=4000)
    srv = pm.Server(max_inflight=16)
    tickets = srv.submit_many([(a, b, p, i) for i, (a, b, p) in enumerate(reqs)])
    assert len(set(tickets)) == len(reqs)
    out = srv.drain()
    assert sorted(c["tag"] for c in out) == list(range(len(reqs)))
    for c in out:
        a, b, p = reqs[c["tag"]]
        assert c["status"] == 0 and same(c["g"], oracle.gcd(a, b, p)), c["tag"]
    ok = reqs[0]
    with pytest.raises(pm.PolyModPError) as e:
        srv.submit_many([(ok[0], ok[1], ok[2], 0), (ok[0], ok[1], 91, 1)])
    assert e.value.status == pm.PM_EMODULUS
    assert srv.pending() == 0
    srv.close()


def _capacity_requests():
    """Instances at the largest served degree (D = 16384) and at the batch
    capacity (17,408 terms), for both block shapes' edges: 4096 terms is the
    256-thread shape's last size, 4097 the 1024-thread shape's first."""
    st = gen.Stream(507)
    cases = []
    for D, dg, p in [(16384, 4096, gen.P_A), (16384, 0, gen.P_B), (17407, 1000, gen.P_C), (17407, 17000, gen.P_A),
                     (4095, 1000, gen.P_B), (4096, 7, gen.P_A)]:
        pl = gen.planted_gcd(D, D - 1, dg, p, st)
        cases.append((oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p), p))
    # uniform pairs of exactly the capacity (coprime with high probability)
    a, b = st.uniform_poly(17407, gen.P_B), st.uniform_poly(17407, gen.P_B)
    cases.append((a, b, gen.P_B))
    return cases


def test_gcd_batch_and_server_at_capacity():
    reqs = _capacity_requests()
    assert max(max(a.size, b.size) for a, b, _ in reqs) == pm.GCD_BATCH_MAX
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=8) as ex:
        want = list(ex.map(lambda r: oracle.gcd(r[0], r[1], r[2], with_info=True), reqs))
    for i, (g, r) in enumerate(pm.gcd_batch([(dev(a), dev(b), p) for a, b, p in reqs])):
        wg, _, stats = want[i]
        assert r["status"] == 0 and same(host(g), wg), i
        assert r["steps"] == stats.steps and r["updates"] == stats.updates, i
    srv = pm.Server()
    srv.submit_many([(a, b, p, i) for i, (a, b, p) in enumerate(reqs)])
    out = srv.drain()
    assert sorted(c["tag"] for c in out) == list(range(len(reqs)))
    for c in out:
        wg, _, stats = want[c["tag"]]
        assert c["status"] == 0 and same(c["g"], wg), c["tag"]
        assert c["steps"] == stats.steps, c["tag"]
    srv.close()


def test_server_admission_waits_for_memory_and_slots():
    reqs = _served_requests(20, 503, lo=500, hi=3000)
    srv = pm.Server(max_inflight=3, arena_words=8192)  # at most a few resident at once
    for i, (a, b, p) in enumerate(reqs):
        srv.submit(a, b, p, tag=i)
    out = srv.drain()
    assert sorted(c["tag"] for c in out) == list(range(20))
    for c in out:
        a, b, p = reqs[c["tag"]]
        assert c["status"] == 0 and same(c["g"], oracle.gcd(a, b, p))
    big = np.ones(9000, dtype=np.uint32)
    with pytest.raises(pm.PolyModPError) as e:
        srv.submit(big, big, gen.P_A)
    assert e.value.status == pm.PM_ENOMEM
    with pytest.raises(pm.PolyModPError) as e:
        srv.submit(big[:5], big[:3], 91)
    assert e.value.status == pm.PM_EMODULUS
    srv.close()


def _division_requests(count, seed, lo=8, hi=6000):
    """Division requests: a of degree D log-uniform in [lo, hi], b of a
    degree uniform in [0, D], uniform residues, three primes."""
    st = gen.Stream(seed)
    reqs = []
    for _ in range(count):
        p = gen.PRIMES[st.index(3)]
        D = st.log_uniform_int(lo, hi)
        db = st.uniform_int(0, D)
        reqs.append((st.uniform_poly(D, p), st.uniform_poly(db, p), p))
    return reqs


def _check_division(c, a, b, p):
    wq, wr = oracle.divrem(a, b, p)
    assert c["status"] == 0 and c["op"] == pm.PM_OP_DIVREM, c["tag"]
    assert same(c["q"], wq) and same(c["r"], wr), c["tag"]
    nzb = np.nonzero(b)[0]
    db1 = int(nzb[-1]) + 1 if nzb.size else 0  # deg b + 1: high zeros do not count
    assert c["steps"] == wq.size and c["updates"] == wq.size * db1, c["tag"]


def test_server_division_requests():
    # both worker shapes (up to 4096 terms on the 256-thread blocks), the
    # capacity, long and short quotients, deg a < deg b, constant divisors,
    # and division requests with high zeros
    reqs = _division_requests(40, 511) + _division_requests(4, 512, lo=5000, hi=17407)
    st = gen.Stream(513)
    p = gen.P_B
    a = st.uniform_poly(17406, p)
    z = np.zeros(30, dtype=np.uint32)
    reqs += [(a, st.uniform_poly(8000, p), p), (a, st.uniform_poly(0, p), p), (a[:4096], a[:4096], p),
             (a[:100], st.uniform_poly(3000, p), p), (np.zeros(0, np.uint32), a[:50], p),
             (np.concatenate([a[:700], z]), np.concatenate([a[:300], z]), p),
             (st.uniform_poly(4095, 2), st.uniform_poly(2000, 2), 2)]
    srv = pm.Server(large_blocks=128)  # the small requests on 256-thread blocks
    srv.submit_many([(x, y, q, i, True) for i, (x, y, q) in enumerate(reqs)])
    out = srv.drain()
    assert sorted(c["tag"] for c in out) == list(range(len(reqs)))
    for c in out:
        _check_division(c, *reqs[c["tag"]])
    # device errors come back in the completion; b = 0 given empty on the host
    bad = a[:60].copy()
    bad[9] = p + 3
    srv.submit_many([(a[:60], np.zeros(8, np.uint32), p, 0, True), (bad, a[:20], p, 1, True)])
    st_by_tag = {c["tag"]: c["status"] for c in srv.drain()}
    assert st_by_tag == {0: pm.PM_EDIVZERO, 1: pm.PM_ERANGE}
    with pytest.raises(pm.PolyModPError) as e:
        srv.submit(a[:60], np.zeros(0, np.uint32), p, divrem=True)
    assert e.value.status == pm.PM_EDIVZERO
    srv.close()


def test_server_gcd_and_division_same_alone_and_in_the_mix():
    gcds = _served_requests(30, 514) + _served_requests(3, 515, lo=5000, hi=16000)
    divs = _division_requests(30, 516) + _division_requests(2, 517, lo=5000, hi=16000)
    mix = [(a, b, p, False) for a, b, p in gcds] + [(a, b, p, True) for a, b, p in divs]
    # gcds and divisions interleaved in submission order
    ng = len(gcds)
    idx = [j for pair in zip(range(ng), range(ng, len(mix))) for j in pair]
    idx += [j for j in range(len(mix)) if j not in set(idx)]
    srv = pm.Server()
    done = {}
    # three waves while polling: later requests join a GPU already working
    for w in range(3):
        srv.submit_many([(mix[i][0], mix[i][1], mix[i][2], i, mix[i][3]) for i in idx[w::3]])
        for c in srv.poll():
            done[c["tag"]] = c
    for c in srv.drain():
        done[c["tag"]] = c
    assert len(done) == len(mix)
    for i, (a, b, p, div) in enumerate(mix):
        if div:
            _check_division(done[i], a, b, p)
        else:
            assert done[i]["status"] == 0 and same(done[i]["g"], oracle.gcd(a, b, p)), i
    srv.close()
    # alone: a fresh server per request, results and counts identical
    for i in [0, len(gcds) - 1, len(gcds), len(mix) - 1]:
        a, b, p, div = mix[i]
        solo = pm.Server()
        solo.submit(a, b, p, tag=i, divrem=div)
        c = solo.drain()[0]
        key = ("q", "r") if div else ("g",)
        assert all(same(c[k], done[i][k]) for k in key) and c["steps"] == done[i]["steps"], i
        solo.close()


def test_server_worker_shapes_give_identical_results():
    # every request on the 1024-thread worker (the default), a split that
    # gives the small requests to 256-thread blocks on 64 CUs, few blocks of
    # each shape, and the inputs read from pinned host memory instead of
    # the device arena: the same results
    reqs = _served_requests(24, 519, lo=30, hi=9000)
    divs = _division_requests(8, 520, lo=30, hi=9000)
    subs = [(a, b, p, i, False) for i, (a, b, p) in enumerate(reqs)]
    subs += [(a, b, p, len(reqs) + i, True) for i, (a, b, p) in enumerate(divs)]
    results = []
    for opts in [dict(), dict(large_blocks=192), dict(large_blocks=4, small_blocks=6), dict(staging=2)]:
        srv = pm.Server(**opts)
        srv.submit_many(subs)
        out = {c["tag"]: c for c in srv.drain()}
        srv.close()
        results.append(out)
    for i, (a, b, p) in enumerate(reqs):
        assert same(results[0][i]["g"], oracle.gcd(a, b, p)), i
    for out in results[1:]:
        for t, c in results[0].items():
            keys = ("q", "r") if c["op"] == pm.PM_OP_DIVREM else ("g",)
            assert all(same(out[t][k], c[k]) for k in keys) and out[t]["steps"] == c["steps"], t


# ------------------------------------------------------------- radix sort
def _sort_inputs(st, n, kind):
    if kind == "uniform":
        return st.raw(n).astype(np.uint32) if n else np.zeros(0, np.uint32)
    if kind == "few":
        return (st.raw(n) % np.uint64(4)).astype(np.uint32)
    if kind == "sorted":
        return np.sort(st.raw(n).astype(np.uint32))
    if kind == "reversed":
        return np.sort(st.raw(n).astype(np.uint32))[::-1].copy()
    return np.full(n, 0xDEADBEEF, dtype=np.uint32)


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_radix_sort_matches_oracle(s):
    # keys and values bit-exact against the oracle's stable LSD sort: empty,
    # one key, ragged tails around the 4096-key tile, several tiles, every
    # digit width, key_bits below 32 (only the low bits order the keys)
    st = gen.Stream(400 + s)
    for n, kind, bits in [(0, "uniform", 32), (1, "uniform", 32), (100, "few", 32), (4095, "uniform", 32),
                          (4096, "sorted", 32), (4097, "reversed", 32), (50000, "uniform", 20),
                          (70001, "few", 7), (12288, "equal", 32), (200003, "uniform", 32)]:
        keys = _sort_inputs(st, n, kind)
        vals = st.raw(n).astype(np.uint32) if n else np.zeros(0, np.uint32)
        ko, vo = pm.radix_sort(dev(keys), dev(vals), s=s, key_bits=bits)
        wk, wv = oracle.radix_sort(keys, vals, bits, s)
        assert same(host(ko), wk) and same(host(vo), wv), (s, n, kind, bits)
        ko2, vo2 = pm.radix_sort(dev(keys), None, s=s, key_bits=bits)
        assert vo2 is None and same(host(ko2), wk), (s, n, kind, "keys only")


def test_radix_sort_workload_64m_properties():
    # the 2^26-key workload of the sweep, at the default s: sorted, a
    # permutation (values = input positions), stable (equal keys keep order)
    import torch
    n = 1 << 26
    st = gen.Stream(gen.SEED_BASE + 9)
    keys = st.raw(n).astype(np.uint32)
    k = dev(keys)
    idx = torch.arange(n, dtype=torch.int32, device="cuda")
    ko, vo = pm.radix_sort(k, idx)
    hk, hv = host(ko), host(vo)
    assert np.all(hk[1:] >= hk[:-1])
    assert np.array_equal(np.sort(hv), np.arange(n, dtype=np.uint32))
    assert np.array_equal(keys[hv], hk)
    eq = hk[1:] == hk[:-1]
    assert np.all(hv[1:][eq] > hv[:-1][eq])


def test_radix_sort_rejects_bad_arguments():
    import torch
    k = dev(np.arange(10, dtype=np.uint32))
    out = torch.empty(10, dtype=torch.int32, device="cuda")
    for kw in [dict(s=11), dict(key_bits=0), dict(key_bits=33)]:
        with pytest.raises(pm.PolyModPError) as e:
            pm.radix_sort(k, **kw)
        assert e.value.status == pm.PM_EINVAL
    with pytest.raises(pm.PolyModPError) as e:
        pm.radix_sort(k, out=(k, None))
    assert e.value.status == pm.PM_EINVAL
    ko, _ = pm.radix_sort(k, out=(out, None))
    assert same(host(ko), np.arange(10, dtype=np.uint32))
