"""The boundary's newer entry points against the oracle, through the C ABI:

* p = 2 in every gcd entry point (the REDC steps with the p = 2 constant);
* the asynchronous division and gcd (results and status in device memory);
* a caller workspace: asynchronous products captured in a graph with no
  warm-up call, replayed with eager work between the replays, and the
  asynchronous division and gcd on the same workspace, allocating nothing;
* a pool that grows after a graph captured its scratch: the graph still
  replays correctly (outgrown buffers are retired, not freed)."""
import numpy as np
import pytest

import oracle
import paper_1402_0264_amd as pm
from paper_1402_0264_amd import gen
from tests.test_gpu_trace import oracle_walk

pytestmark = pytest.mark.gpu


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


def same(x, y):
    return np.array_equal(np.asarray(x, dtype=np.uint32), np.asarray(y, dtype=np.uint32))


def _planted(st, da, db, dg, p):
    pl = gen.planted_gcd(da, db, dg, p, st)
    return oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)


# ------------------------------------------------------------------ p = 2
P2_SHAPES = [(5, 3, 0), (40, 40, 3), (100, 60, 20), (60, 100, 59), (700, 699, 10), (2000, 1999, 300),
             (2000, 100, 30), (120, 1500, 0), (5000, 4999, 40)]


def test_gcd_at_p2_matches_oracle():
    p = 2
    st = gen.Stream(gen.SEED_BASE + 401)
    z = np.zeros(0, dtype=np.uint32)
    cases = [_planted(st, da, db, dg, p) + ((da, db, dg),) for da, db, dg in P2_SHAPES]
    x = st.uniform_poly(30, p)
    cases += [(z, z, "0,0"), (x, z, "x,0"), (z, x, "0,x"), (x, x, "x,x"), (x, np.ones(1, np.uint32), "x,1")]
    for a, b, tag in cases:
        want, degs, stats = oracle.gcd(a, b, p, with_info=True)
        assert same(host(pm.gcd(dev(a), dev(b), p)), want), tag
        got = pm.last_gcd_stats()
        assert (got["steps"], got["updates"]) == (stats.steps, stats.updates), tag
        g, d = pm.gcd_degrees(dev(a), dev(b), p)
        assert same(host(g), want) and list(d) == list(degs), tag
        g, s, t = pm.xgcd(dev(a), dev(b), p)
        wg, ws, wt = oracle.xgcd(a, b, p)
        assert same(host(g), wg) and same(host(s), ws) and same(host(t), wt), tag


def test_checkpoints_at_p2():
    p = 2
    st = gen.Stream(gen.SEED_BASE + 402)
    ks = [0, 1, 2, 63, 64, 65, 300, 1999, 10 ** 6]
    for da, db, dg in [(300, 299, 20), (1500, 1499, 0), (1100, 700, 30)]:
        a, b = _planted(st, da, db, dg, p)
        want = oracle_walk(a, b, p, ks)
        for k in ks:
            x, y, taken = pm.euclid_steps(dev(a), dev(b), p, k)
            assert (host(x).tolist(), host(y).tolist(), taken) == want[k], (da, db, k)


def test_gcd_batch_at_p2_and_mixed_primes():
    st = gen.Stream(gen.SEED_BASE + 403)
    pairs = []
    for i, (da, db, dg) in enumerate([(300, 299, 20), (4000, 3999, 100), (5000, 4999, 7), (64, 63, 0), (2, 1, 0)]):
        for p in (2, gen.P_A):
            a, b = _planted(st, da, db, dg, p)
            pairs.append((dev(a), dev(b), p, a, b))
    res = pm.gcd_batch([(a, b, p) for a, b, p, _, _ in pairs])
    for (g, r), (_, _, p, a, b) in zip(res, pairs):
        assert r["status"] == 0 and same(host(g), oracle.gcd(a, b, p)), (p, a.size)


# -------------------------------------------------------- async division
def _divrem_async(a, b, p, q_cap=None, r_cap=None):
    import torch
    na, nb = a.size, b.size
    q_cap = max(na - nb + 1, 0) + 3 if q_cap is None else q_cap
    r_cap = min(na, nb - 1) + 2 if r_cap is None else r_cap
    q = torch.full((max(q_cap, 1),), -1, dtype=torch.int32, device="cuda")[:q_cap]
    r = torch.full((max(r_cap, 1),), -1, dtype=torch.int32, device="cuda")[:r_cap]
    d = torch.full((2,), -9, dtype=torch.int64, device="cuda")
    s = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    pm.divrem_async(dev(a) if na else torch.empty(0, dtype=torch.int32, device="cuda"), dev(b), p, q, r,
                    d[0:1], d[1:2], s)
    torch.cuda.synchronize()
    return host(q), host(r), int(d[0].item()), int(d[1].item()), int(s.item())


DIV_SHAPES = [(1, 1), (10, 1), (10, 3), (100, 99), (500, 17), (300, 300), (3, 10), (2049, 2048), (3000, 1100),
              (9000, 7), (20000, 9000), (65536, 32768), (32769, 32768), (700, 2)]


@pytest.mark.parametrize("p", [gen.P_A, gen.P_B, 3, 2])
def test_divrem_async_matches_oracle(p):
    st = gen.Stream(gen.SEED_BASE + 404 + p % 997)
    for na, nb in DIV_SHAPES:
        a, b = st.uniform_poly(na - 1, p), st.uniform_poly(nb - 1, p)
        wq, wr = oracle.divrem(a, b, p)
        q, r, nq, nr, status = _divrem_async(a, b, p)
        assert status == 0 and nq == wq.size and nr == wr.size, (p, na, nb, status, nq, nr)
        assert same(q[:nq], wq) and same(r[:nr], wr), (p, na, nb)
        mu_plan = max(na - nb + 1, 0)
        assert not q[nq:mu_plan].any(), "the quotient is zeroed up to na - nb + 1"
        assert (q[mu_plan:] == 0xFFFFFFFF).all() and (r[min(na, nb - 1):] == 0xFFFFFFFF).all(), "written past"


def test_divrem_async_high_zeros_and_errors():
    import torch
    p = gen.P_C
    st = gen.Stream(gen.SEED_BASE + 405)
    a, b = st.uniform_poly(900, p), st.uniform_poly(300, p)
    z = np.zeros(40, dtype=np.uint32)
    # high zeros of a are allowed, down to deg a < deg b
    for x in (np.concatenate([a, z]), np.concatenate([a[:200], np.zeros(500, np.uint32)]), np.zeros(400, np.uint32)):
        wq, wr = oracle.divrem(x, b, p)
        q, r, nq, nr, status = _divrem_async(x, b, p)
        assert status == 0 and (nq, nr) == (wq.size, wr.size) and same(q[:nq], wq) and same(r[:nr], wr)
    # a divisor given with a zero top coefficient is refused on the device
    q, r, nq, nr, status = _divrem_async(a, np.concatenate([b, z]), p)
    assert status == pm.PM_EINVAL and nq == 0 and nr == 0
    bad = a.copy()
    bad[17] = p
    assert _divrem_async(bad, b, p)[4] == pm.PM_ERANGE
    with pytest.raises(pm.PolyModPError) as e:
        pm.divrem_async(dev(a), torch.empty(0, dtype=torch.int32, device="cuda"), p,
                        torch.empty(901, dtype=torch.int32, device="cuda"),
                        torch.empty(901, dtype=torch.int32, device="cuda"))
    assert e.value.status == pm.PM_EDIVZERO


# ------------------------------------------------------------- async gcd
def test_gcd_async_matches_oracle():
    import torch
    st = gen.Stream(gen.SEED_BASE + 406)
    z = np.zeros(0, dtype=np.uint32)
    for p in (gen.P_A, gen.P_B, 5, 2):
        cases = [_planted(st, da, db, dg, p) for da, db, dg in [(300, 299, 20), (3000, 2999, 500), (1200, 1000, 30),
                                                                  (400, 1000, 10), (64, 0, 0)]]
        x = st.uniform_poly(77, p)
        cases += [(z, z), (x, z), (z, x)]
        for a, b in cases:
            want = oracle.gcd(a, b, p)
            cap = max(a.size, b.size, 1)
            g = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
            d = torch.full((1,), -9, dtype=torch.int64, device="cuda")
            s = torch.full((1,), 77, dtype=torch.int32, device="cuda")
            empty = torch.empty(0, dtype=torch.int32, device="cuda")
            pm.gcd_async(dev(a) if a.size else empty, dev(b) if b.size else empty, p, g, d, s)
            torch.cuda.synchronize()
            assert int(s.item()) == 0 and int(d.item()) == want.size, (p, a.size, b.size)
            assert same(host(g)[:want.size], want), (p, a.size, b.size)
    a, b = _planted(st, 500, 499, 5, gen.P_A)
    a[3] = gen.P_A + 1
    g = torch.empty(500, dtype=torch.int32, device="cuda")
    s = torch.zeros(1, dtype=torch.int32, device="cuda")
    pm.gcd_async(dev(a), dev(b), gen.P_A, g, None, s)
    torch.cuda.synchronize()
    assert int(s.item()) == pm.PM_ERANGE


# ------------------------------------------------- workspace and capture
def test_workspace_capture_without_warmup_then_async_division_and_gcd():
    import torch
    p = gen.P_A
    st = gen.Stream(gen.SEED_BASE + 407)
    # the matrix cores (share partial sums) and the VALU tiles (rows of M)
    shapes = [(20000, 9000), (3001, 2500)]
    pairs = [(st.uniform_poly(na - 1, p), st.uniform_poly(nb - 1, p)) for na, nb in shapes]
    da, db = st.uniform_poly(65535, p), st.uniform_poly(32767, p)
    ga, gb = _planted(st, 6000, 5999, 700, p)
    words = max([pm.workspace_size(pm.PM_OP_MUL, na, nb) for na, nb in shapes] +
                [pm.workspace_size(pm.PM_OP_DIVREM, da.size, db.size),
                 pm.workspace_size(pm.PM_OP_GCD, ga.size, gb.size)])
    ws = torch.zeros(words, dtype=torch.int32, device="cuda")
    side = torch.cuda.Stream()
    pm.set_workspace(ws, stream=side)
    try:
        ins = [(dev(a), dev(b)) for a, b in pairs]
        outs = [torch.full((a.size + b.size - 1,), -1, dtype=torch.int32, device="cuda") for a, b in pairs]
        d_nf = torch.zeros(len(pairs), dtype=torch.int64, device="cuda")
        d_st = torch.full((len(pairs),), 7, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):  # the first call of the stream is inside the capture
            for i, (x, y) in enumerate(ins):
                pm.mul_async(x, y, p, outs[i], d_nf[i:i + 1], d_st[i:i + 1])
        want = [oracle.mul(a, b, p) for a, b in pairs]
        for rep in range(3):
            for o in outs:
                o.fill_(-1)
            d_st.fill_(7)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert d_st.tolist() == [0] * len(pairs), rep
            for o, w in zip(outs, want):
                assert same(host(o), w), rep
            # eager work between replays, on the default stream's own pool
            pm.mul(dev(pairs[1][0]), dev(pairs[1][1]), p)
        # the asynchronous division and gcd on the same workspace
        with torch.cuda.stream(side):
            q = torch.empty(da.size - db.size + 1, dtype=torch.int32, device="cuda")
            r = torch.empty(db.size - 1, dtype=torch.int32, device="cuda")
            g = torch.empty(ga.size, dtype=torch.int32, device="cuda")
            lens = torch.zeros(3, dtype=torch.int64, device="cuda")
            sts = torch.full((2,), 7, dtype=torch.int32, device="cuda")
            pm.divrem_async(dev(da), dev(db), p, q, r, lens[0:1], lens[1:2], sts[0:1], stream=side)
            pm.gcd_async(dev(ga), dev(gb), p, g, lens[2:3], sts[1:2], stream=side)
        side.synchronize()
        wq, wr = oracle.divrem(da, db, p)
        wg = oracle.gcd(ga, gb, p)
        assert sts.tolist() == [0, 0] and lens.tolist() == [wq.size, wr.size, wg.size]
        assert same(host(q), wq) and same(host(r)[:wr.size], wr) and same(host(g)[:wg.size], wg)
        # a call that needs more than the workspace is refused, allocating nothing
        big = st.uniform_poly(150000, p)
        f = torch.empty(2 * big.size - 1, dtype=torch.int32, device="cuda")
        if pm.workspace_size(pm.PM_OP_MUL, big.size, big.size) > words:
            with pytest.raises(pm.PolyModPError) as e:
                pm.mul_async(dev(big), dev(big), p, f, d_nf[0:1], d_st[0:1], stream=side)
            assert e.value.status == pm.PM_ENOMEM
    finally:
        pm.set_workspace(None, stream=side)
        torch.cuda.synchronize()


def test_pool_growth_keeps_a_captured_graph_valid():
    import torch
    p = gen.P_B
    st = gen.Stream(gen.SEED_BASE + 408)
    small = (st.uniform_poly(3000, p), st.uniform_poly(2499, p))   # VALU tiles, 20 b-chunks
    large = (st.uniform_poly(19999, p), st.uniform_poly(8999, p))  # the matrix cores: a larger scratch
    side = torch.cuda.Stream()
    xs, ys = dev(small[0]), dev(small[1])
    f = torch.empty(small[0].size + small[1].size - 1, dtype=torch.int32, device="cuda")
    d_nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    d_st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(side):
        pm.mul_async(xs, ys, p, f, d_nf, d_st, stream=side)  # sizes the stream's pool
    side.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        pm.mul_async(xs, ys, p, f, d_nf, d_st)
    # a larger product on the same stream grows its pool
    with torch.cuda.stream(side):
        fl = pm.mul(dev(large[0]), dev(large[1]), p, stream=side)
    side.synchronize()
    assert same(host(fl), oracle.mul(large[0], large[1], p))
    want = oracle.mul(small[0], small[1], p)
    for rep in range(3):
        f.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert int(d_st.item()) == 0 and same(host(f), want), rep
        with torch.cuda.stream(side):
            pm.mul(dev(large[0]), dev(large[1]), p, stream=side)
        side.synchronize()


def test_kernel_timing_records_launches_and_leaves_results_unchanged():
    """pm_timing_*: with timing on, every matrix-core product records one
    mulx_kernel launch (events carried by the launch itself) and a division
    its flow kernel (events recorded around it), each with a positive
    duration; the timed results equal the oracle's, and with timing off
    nothing more is recorded."""
    import torch
    p = gen.P_A
    st = gen.Stream(gen.SEED_BASE + 409)
    a, b = st.uniform_poly(9000, p), st.uniform_poly(7001, p)
    da, db = dev(a), dev(b)
    want = oracle.mul(a, b, p)
    try:
        pm.timing_reset()
        pm.timing_enable(True)
        try:
            q, r = pm.divrem(da, db, p)  # default engine: its remainder product takes the VALU tiles
            pm.set_params(mul_engine=pm.MUL_MFMA)
            outs = [pm.mul(da, db, p) for _ in range(3)]
        finally:
            pm.timing_enable(False)
        torch.cuda.synchronize()
        n, ms = pm.timing_read("mulx_kernel")
        assert n == 3 and ms > 0.0, (n, ms)
        n_div, ms_div = pm.timing_read("divrem_flow_kernel")
        assert n_div == 1 and ms_div > 0.0, (n_div, ms_div)
        for f in outs:
            assert same(host(f), want)
        wq, wr = oracle.divrem(a, b, p)
        assert same(host(q), wq) and same(host(r), wr)
        pm.mul(da, db, p)  # timing off: not recorded
        torch.cuda.synchronize()
        assert pm.timing_read("mulx_kernel")[0] == 3
        pm.timing_reset()
        assert pm.timing_read("mulx_kernel") == (0, 0.0)
    finally:
        pm.set_params()
