"""Host logic of the per-query fixed-point plan (gs_query_plan_host), on the CPU.

The doc-tiled kernels sum w_q(t) * w_d(t) (Sec. 4.1) in integer units of 2^-F:
each product rounds to the nearest unit (ties to even: the fp64 FMA
qd * w_d + 2^52 with every product below 2^51 units), the units are summed
exactly, and the sum is converted to fp32. The plan must (1) keep every sum inside
its accumulator (2^63 for fp32, 2^32 for bf16), (2) bound the error of every
document's sum by abs_err, and (3) set the wide-range limit so that every score
at or above it is within 2^-18 (plus the final fp32 rounding) of the exact one.
Exact rational arithmetic (fractions.Fraction) stands in for the kernel's
integer sums here; nothing is taken from the library but the plan.
"""
from fractions import Fraction

import numpy as np
import pytest

RHO = {"fp32": 2.0 ** -18, "bf16": 2.0 ** -12}
ACC_LIMIT = {"fp32": 2 ** 63, "bf16": 2 ** 32}


def _gs():
    import paper_2606_26441_amd as gs
    return gs


def _bf16(x):
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32)


def _fx_sum(qw, dw, F):
    """Integer units of one document: each exact product rounded half to even."""
    s = 0
    for a, b in zip(qw, dw):
        s += round(Fraction(float(a)) * Fraction(float(b)) * Fraction(2) ** F)
    return s


def _instance(rng, m, lo_exp, hi_exp, n_docs=40):
    """Query weights and, per term, a posting list of weights (log-uniform over [10^lo, 10^hi])."""
    qw = (10.0 ** rng.uniform(lo_exp, hi_exp, size=m)).astype(np.float32)
    lists = [(10.0 ** rng.uniform(lo_exp, hi_exp, size=n_docs)).astype(np.float32) for _ in range(m)]
    return qw, lists


def _check_plan(gs, precision, qw, lists, rng, n_docs=40):
    m = len(qw)
    stored = [(_bf16(w) if precision == "bf16" else w) for w in lists]
    tmax = np.array([w.max() for w in stored], np.float32)
    tmin = np.array([w[w > 0].min() if np.any(w > 0) else np.inf for w in stored], np.float32)
    F, abs_err, lim = gs.query_plan_host(precision, qw, tmax, tmin)
    unit = Fraction(2) ** -F
    # documents: random subsets of the query terms, weights from each term's list
    for d in range(n_docs):
        mask = rng.random(m) < 0.6
        mask[rng.integers(m)] = True
        idx = np.flatnonzero(mask)
        dw = [stored[t][d] for t in idx]
        units = _fx_sum(qw[idx], dw, F)
        assert 0 <= units < ACC_LIMIT[precision], "accumulator overflow"
        exact = sum(Fraction(float(qw[t])) * Fraction(float(w)) for t, w in zip(idx, dw))
        err = abs(units * unit - exact)
        assert err <= Fraction(abs_err), "fixed-point error above abs_err"
        got = float(np.float32(float(units * unit)))  # the kernel's fp32 score
        if exact > 0 and got >= lim:
            rel = abs(Fraction(got) - exact) / exact
            assert rel <= Fraction(RHO[precision]) * (1 + Fraction(1, 10 ** 6)) + Fraction(2) ** -23, \
                "score above the wide-range limit misses the relative budget"
    return F, abs_err, lim


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("m", [1, 3, 30, 256])
def test_plan_bounds_on_ordinary_weights(precision, m):
    # weights like the synthetic workload's (0.005 .. 3): the limit is 0 for fp32, i.e. no
    # query can ever need the fp64 pass
    gs = _gs()
    rng = np.random.default_rng(m)
    qw, lists = _instance(rng, m, np.log10(0.005), np.log10(3.0))
    F, abs_err, lim = _check_plan(gs, precision, qw, lists, rng)
    if precision == "fp32":
        assert lim == 0.0


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("m", [2, 8, 64, 256])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plan_bounds_on_wide_range_weights(precision, m, seed):
    # weights spread over 12 orders of magnitude: the bound must still hold, and the limit
    # becomes positive (some score may be too small for the fixed-point error)
    gs = _gs()
    rng = np.random.default_rng(100 * m + seed)
    qw, lists = _instance(rng, m, -12.0, np.log10(3.0))
    F, abs_err, lim = _check_plan(gs, precision, qw, lists, rng)
    assert lim > 0.0


def test_plan_of_the_three_scale_query():
    # query {3.0, 1e-5, 1e-9} over lists whose weights lie near 1, 1e-5 and 1e-9: the largest
    # product (9) sets the scale, the smallest positive one (~5e-19) lies far below the limit
    gs = _gs()
    qw = np.array([3.0, 1e-5, 1e-9], np.float32)
    tmax = np.array([3.0, 2e-5, 2e-9], np.float32)
    tmin = np.array([0.5, 5e-6, 5e-10], np.float32)
    F, abs_err, lim = gs.query_plan_host("fp32", qw, tmax, tmin)
    assert 9.0 * 2.0 ** F < 2.0 ** 51 <= 2 * 9.0 * 2.0 ** F  # the largest product just below 2^51 units
    assert lim > 1e-10 > 5e-19  # B-only and C-only scores both fall below the limit
    # without the small terms the same scale clears every positive score
    _, _, lim2 = gs.query_plan_host("fp32", qw[:1], tmax[:1], tmin[:1])
    assert lim2 == 0.0


def test_plan_rejects_bad_input():
    gs = _gs()
    with pytest.raises(gs.GsError):
        gs.query_plan_host("u8", [1.0], [1.0], [1.0])
    with pytest.raises(gs.GsError):
        gs.query_plan_host("fp32", [-1.0], [1.0], [1.0])
    with pytest.raises(gs.GsError):
        gs.query_plan_host("fp32", [1.0], [1.0], [0.0])
