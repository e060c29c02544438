"""The model evaluator (paper_1402_0264_amd.mmm) rebuilt from the printed
N, L, C of each algorithm reproduces the running-time ratios and thresholds
the paper prints (tests/golden/paper_model.json)."""
import json
import math
import os

import sympy as sp

from paper_1402_0264_amd import mmm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_model.json")))
n, m, U, Z, s, ell = sp.symbols("n m U Z s l", positive=True)
c_ = sp.symbols("c", positive=True)


def _expr(key):
    return sp.sympify(GOLD[key]["expr"], locals={"n": n, "U": U, "Z": Z, "s": s, "l": ell, "log": sp.log})


def test_division_ratio_matches_printed():
    T1 = mmm.div_time_naive(n, m, U, Z / 2)
    Ts = mmm.div_time(n, m, Z / 7, U)
    assert sp.simplify(T1 / Ts - _expr("division_R")) == 0


def test_division_work_and_overhead_ratios():
    # W_1, W_s, O_1, O_s as printed in Sec. 3.1 and 3.2, at l = Z/2, s = Z/7
    W1 = (n - m + 1) * m * (2 * ell + 1) / ell
    Ws = (n - m + 1) * m * (9 * s + 1) / (4 * s)
    O1 = 5 * (n - m + 1) * m * U / ell
    Os = 9 * (n - m + 1) * m * U / (2 * s ** 2)
    sub = {ell: Z / 2, s: Z / 7}
    assert sp.simplify((W1 / Ws).subs(sub) - _expr("division_work_ratio")) == 0
    assert sp.simplify((O1 / Os).subs(sub) - _expr("division_overhead_ratio")) == 0


def test_gcd_ratio_matches_printed():
    T1 = mmm.gcd_time_naive(n, n, U, Z / 2)
    Ts = mmm.gcd_time(n, n, Z / 6, U)
    assert sp.simplify(T1 / Ts - _expr("gcd_R")) == 0
    assert sp.simplify(sp.limit(_expr("gcd_R"), n, sp.oo) - _expr("gcd_R_limit")) == 0


def test_mul_ratio_matches_printed():
    printed = _expr("mul_R")
    for nv, sv, uv in [(4096, 4, 20), (65536, 16, 3), (1000, 7, 0.5)]:
        got = mmm.mul_time(nv, nv, 1, uv) / mmm.mul_time(nv, nv, sv, uv)
        want = printed.subs({n: nv, s: sv, U: uv})
        assert abs(float(got) - float(want)) < 1e-9 * float(want)
        assert abs(mmm.mul_ratio_printed(nv, sv, uv) - float(want)) < 1e-9 * float(want)


def test_thresholds():
    # R > 1 iff Z > threshold, for every positive U
    for uv in [0.5, 3, 20, 600]:
        zd = GOLD["division_threshold_Z"]["value"]
        zg = GOLD["gcd_threshold_Z"]["value"]
        assert mmm.div_ratio_printed(zd * 1.01, uv) > 1 > mmm.div_ratio_printed(zd * 0.99, uv)
        lim = sp.lambdify((Z, U), _expr("gcd_R_limit"))
        assert lim(zg * 1.01, uv) > 1 > lim(zg * 0.99, uv)


def test_model_directions_on_mi355x_constants():
    r = mmm.predicted_ranges()
    assert r["mul"]["argmin_s"] == 1                  # product: s as small as possible
    assert r["div"]["argmin_s"] == 256                # division: the largest feasible s (3s <= 1024)
    assert r["gcd"]["argmin_s"] == 256                # gcd: s* beyond the feasible range
    assert r["gcd"]["s_star_real"] > 256
    for s_ in [1, 2, 8, 64]:
        assert mmm.mul_time(65536, 65536, s_, 20) < mmm.mul_time(65536, 65536, 2 * s_, 20)
    assert math.isclose(mmm.U_THROUGHPUT, 64 / (8e12 / 4 / 256 / 2.4e9))


def test_sort_ratio_matches_printed():
    # T_1/T_s from the printed N_s, L_s, C_s (Corollary 1, one block per tile
    # of 4l keys) is the printed R, for every n, c, l, U and s
    lg = sp.log(ell, 2)

    def T(sv):
        N = (c_ / sv) * (1 / (2 * ell) + 2 ** sv / (8 * ell ** 2)) * n
        L = 5 * c_ / sv
        C = sv * (41 + 8 * lg) + 12 + 9 * U
        return (N / (n / (4 * ell)) + L) * C
    assert sp.simplify(T(1) / T(s) - _expr("sort_R")) == 0
    for nv, cv, sv, lv, uv in [(1 << 26, 32, 8, 256, 19.7), (1000, 20, 3, 64, 2.0)]:
        got = mmm.sort_time(nv, cv, 1, uv, lv) / mmm.sort_time(nv, cv, sv, uv, lv)
        assert abs(got - mmm.sort_ratio_printed(sv, uv, lv)) < 1e-9 * got
        want = float(_expr("sort_R").subs({ell: lv, s: sv, U: uv}))
        assert abs(got - want) < 1e-9 * got


def test_sort_overhead_ratio_and_threshold():
    # O_s as printed; O_1/O_s tends to the printed ratio as n grows, and the
    # leading-term quotient at s = log2 l exceeds 1 exactly below the
    # printed threshold l < 2^(15.75 U)
    def O(sv):
        return c_ * U * (sp.Rational(9, 2) / (sv * ell) * n + 17 * 2 ** sv / (16 * sv * ell ** 2) * n - 1 / sv)
    lim = sp.limit(O(1) / O(s), n, sp.oo)
    assert sp.simplify(lim - _expr("sort_overhead_ratio")) == 0
    q = sp.lambdify((ell, U), _expr("sort_leading_quotient"))
    t = GOLD["sort_threshold_log2_l_over_U"]["value"]
    for uv in [0.5, 1, 4]:
        edge = 2 ** (t * uv)
        assert q(edge * 0.9, uv) > 1 > q(edge * 1.1, uv)
