"""Parity of the gcd's intermediate state with the oracle (Sec. 6, Alg. 9):

* the degree sequence of the remainder sequence, rebuilt from the kernel's
  own step log (poly_gcd_modp_degrees), equals the oracle's exactly: on the
  degree-32768 workload, on Table 2's nine (n, m) pairs, and at p = 3 and 5
  where remainders often lose several degrees at once;
* checkpoints: after k division steps (poly_euclid_steps_modp) the pair,
  made monic, equals the oracle's naive Euclidean step walked k times, for
  several k that end inside, at and across chunk boundaries, on one block
  and on the cooperative grid, with steps whose shift exceeds a chunk's
  matrix.

The steps are scaled by units on the GPU, so the pair is compared monic
(the canonical representative); degrees and step counts are exact."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1402_0264_amd as pm
from paper_1402_0264_amd import gen

pytestmark = pytest.mark.gpu

TABLE2 = [(2000, 1500), (3000, 2500), (4000, 3500), (5000, 4500), (6000, 5000), (7000, 6000), (8000, 7000),
          (9000, 8000), (10000, 9000)]


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


def check_degrees(a, b, p, tag):
    g, degs = pm.gcd_degrees(dev(a), dev(b), p)
    want_g, want_degs, _ = oracle.gcd(a, b, p, with_info=True)
    assert np.array_equal(host(g), want_g), tag
    assert list(degs) == list(want_degs), (tag, list(degs[:12]), list(want_degs[:12]))
    return want_degs


def test_degree_sequence_gcd_32768():
    pl = gen.gcd_32768()
    p = pl.p
    a, b = oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)
    degs = check_degrees(a, b, p, "gcd_32768")
    assert degs[-2] == 1000


@pytest.mark.parametrize("n,m", TABLE2)
def test_degree_sequence_table2_pairs(n, m):
    # Table 2's shapes: uniform random a of n terms and b of m terms; the
    # degree gap starts the gcd with one Euclidean division
    p = gen.P_A
    st = gen.Stream(gen.SEED_BASE + 40 + TABLE2.index((n, m)))
    a, b = st.uniform_poly(n - 1, p), st.uniform_poly(m - 1, p)
    check_degrees(a, b, p, (n, m))


@pytest.mark.parametrize("p", [3, 5, gen.P_C])
def test_degree_sequence_small_primes(p):
    st = gen.Stream(701 + p % 997)
    skipped = 0
    for da, db in [(40, 39), (40, 40), (300, 299), (700, 650), (1500, 1499), (1200, 1000), (500, 1200),
                   (2000, 100), (64, 63), (3000, 2999)]:
        for rep in range(2):
            a, b = st.uniform_poly(da, p), st.uniform_poly(db, p)
            if rep and da > 50:  # a planted common factor as well
                pl = gen.planted_gcd(da, db, da // 5, p, st)
                a, b = oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)
            degs = check_degrees(a, b, p, (p, da, db, rep))
            skipped += any(x - y > 1 for x, y in zip(degs[1:-2], degs[2:-1]))
    if p < 10:
        assert skipped >= 5


def test_degree_sequence_degenerate():
    p = gen.P_A
    st = gen.Stream(702)
    z = np.zeros(0, dtype=np.uint32)
    x = st.uniform_poly(300, p)
    one = np.array([5], dtype=np.uint32)
    for a, b in [(z, z), (x, z), (z, x), (x, x), (x, one), (one, x), (one, one)]:
        check_degrees(a, b, p, (a.size, b.size))
    # b divides a: the sequence stops after one division
    h = st.uniform_poly(40, p)
    check_degrees(oracle.mul(x, h, p), x, p, "exact")


def _monic(x, p):
    x = [int(v) for v in x]
    while x and x[-1] == 0:
        x.pop()
    if not x:
        return []
    inv = pow(x[-1], p - 2, p)
    return [v * inv % p for v in x]


def oracle_walk(a, b, p, ks):
    """The pair after k naive Euclidean steps of the oracle, for each k in
    ks: {k: (monic a_k, monic b_k, steps taken)}."""
    L = oracle.lib()
    n = max(a.size, b.size, 1)
    A = np.zeros(n, dtype=np.uint32)
    B = np.zeros(n, dtype=np.uint32)
    A[:a.size] = a
    B[:b.size] = b
    da = ctypes.c_int64(int(np.nonzero(A)[0][-1]) if A.any() else -1)
    db = ctypes.c_int64(int(np.nonzero(B)[0][-1]) if B.any() else -1)
    pa = A.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    pb = B.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    out = {}
    taken = 0
    for k in sorted(ks):
        while taken < k:
            if not L.orc_euclid_step(pa, ctypes.byref(da), pb, ctypes.byref(db), p):
                break
            taken += 1
        out[k] = (_monic(A[:da.value + 1], p), _monic(B[:db.value + 1], p), taken)
    return out


KS = [0, 1, 2, 3, 62, 63, 64, 65, 126, 127, 128, 129, 255, 256, 300, 777, 1500, 2999, 10 ** 6]


@pytest.mark.parametrize("p", [gen.P_A, 3, 5])
def test_checkpoints_match_the_oracle_walk(p):
    st = gen.Stream(703 + p % 997)
    cases = []
    for da, db, dg in [(300, 299, 20), (300, 300, 0), (1500, 1499, 100), (1100, 700, 30), (400, 1000, 10),
                       (2000, 1999, 0)]:
        pl = gen.planted_gcd(da, db, dg, p, st)
        cases.append((oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p), (da, db, dg)))
    cases.append((st.uniform_poly(200, p), np.zeros(0, dtype=np.uint32), "b = 0"))
    for a, b, tag in cases:
        want = oracle_walk(a, b, p, KS)
        for k in KS:
            x, y, taken = pm.euclid_steps(dev(a), dev(b), p, k)
            wa, wb, wt = want[k]
            assert taken == wt, (p, tag, k, taken, wt)
            assert host(x).tolist() == wa, (p, tag, k)
            assert host(y).tolist() == wb, (p, tag, k)


def test_checkpoints_invariant_under_s():
    # the same pair after the same steps whatever the chunk length
    p = gen.P_B
    st = gen.Stream(704)
    pl = gen.planted_gcd(900, 899, 50, p, st)
    a, b = oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)
    ks = [5, 100, 513, 1601]
    want = oracle_walk(a, b, p, ks)
    try:
        for s in [1, 7, 64, 128, 256]:
            pm.set_params(gcd_s=s)
            for k in ks:
                x, y, taken = pm.euclid_steps(dev(a), dev(b), p, k)
                assert (host(x).tolist(), host(y).tolist(), taken) == want[k], (s, k)
    finally:
        pm.set_params()
