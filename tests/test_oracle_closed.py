"""Pins of the oracle's closed-interval reading.

Algorithm 1 of the paper tests two intervals with non-strict comparisons
(lower <= other upper on both sides), i.e. closed intervals [lo, hi].  The
closed reading of the oracle (Algorithm 4 with lower-before-upper ties and no
empty regions) is pinned here by things other than itself: the plain
definition (max of the lowers <= min of the uppers) written twice, in C and in
numpy; the 1-D counting identity for closed intervals; hand-worked special
cases; and an exact reduction to the half-open reading on float32 (x <= y iff
x < nextafter(y, +inf) for finite y), which ties the two readings together.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1703_06680_amd import workloads as W


def _f(a):
    return np.asarray(a, dtype=np.float32).reshape(len(a), -1)


def _next_up(hi):
    return np.nextafter(hi, np.float32(np.inf)).astype(np.float32)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_c_bruteforce_closed_equals_numpy_definition(oracle, d):
    for seed in range(20):
        inst = W.tie_heavy(23, 17, d, seed=seed)
        a = (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)
        hit = O.bruteforce_numpy(*a, closed=True)
        k, per, pairs = oracle.bruteforce(*a, closed=True)
        assert k == int(hit.sum())
        assert np.array_equal(pairs, O.pairs_from_matrix(hit))
        assert np.array_equal(per, hit.sum(axis=1).astype(np.int32))


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("family", ["ties", "float"])
def test_sbm_closed_equals_bruteforce_small(oracle, d, family):
    rng = np.random.default_rng(2000 + d)
    for seed in range(150):
        n, m = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        if family == "ties":
            inst = W.tie_heavy(n, m, d, grid=int(rng.integers(2, 15)),
                               max_len=int(rng.integers(0, 6)), seed=seed)
        else:
            inst = W.random_float_boxes(n, m, d, seed=seed)
        a = (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)
        hit = O.bruteforce_numpy(*a, closed=True)
        k, per, pairs = oracle.sbm(*a, closed=True)
        assert k == int(hit.sum()), (family, d, seed)
        assert np.array_equal(pairs, O.pairs_from_matrix(hit)), (family, d, seed)
        assert np.array_equal(per, hit.sum(axis=1).astype(np.int32)), (family, d, seed)


def test_closed_form_1d_closed(oracle):
    """#{s : s.lo <= u.hi} - #{s : s.hi < u.lo} on the tie-heavy grid and on
    the uniform workload, against the closed sweep."""
    for inst in (W.tie_heavy(3000, 2500, 1, grid=400, max_len=5, seed=3),
                 W.uniform_instance(5000, 5000, 1, 1.0, seed=4)):
        a = (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)
        k, per, _ = oracle.sbm(*a, pairs=False, closed=True)
        cf = O.closed_form_1d(*a, closed=True)
        assert np.array_equal(per.astype(np.int64), cf)
        assert k == int(cf.sum())


@pytest.mark.parametrize("d", [1, 2, 3])
def test_closed_is_half_open_with_the_next_float(oracle, d):
    """Closed [lo, hi] matches exactly as half-open [lo, nextafter(hi))."""
    for seed in range(10):
        for inst in (W.tie_heavy(200, 150, d, grid=30, max_len=4, seed=seed),
                     W.random_float_boxes(200, 150, d, seed=seed)):
            ul, uh, sl, sh = inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi
            kc, pc, qc = oracle.sbm(ul, uh, sl, sh, closed=True)
            kh, ph, qh = oracle.sbm(ul, _next_up(uh), sl, _next_up(sh))
            assert kc == kh and np.array_equal(pc, ph) and np.array_equal(qc, qh)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_closed_contains_half_open(oracle, d):
    for seed in range(10):
        inst = W.tie_heavy(60, 50, d, grid=10, max_len=3, seed=seed)
        a = (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)
        _, _, qc = oracle.sbm(*a, closed=True)
        _, _, qh = oracle.sbm(*a)
        closed = set(map(tuple, qc.tolist()))
        assert set(map(tuple, qh.tolist())) <= closed
        # on generic floats (no shared coordinates, no zero sides) they agree
        f = W.uniform_instance(300, 300, d, 50.0, seed=seed)
        b = (f.upd_lo, f.upd_hi, f.sub_lo, f.sub_hi)
        assert oracle.sbm(*b, closed=True)[0] == oracle.sbm(*b)[0]


def test_closed_special_cases(oracle):
    sbm = lambda *a: oracle.sbm(*a, closed=True)[0]  # noqa: E731
    # touching intervals match; gaps do not
    assert sbm(_f([0.0]), _f([5.0]), _f([5.0]), _f([10.0])) == 1
    assert sbm(_f([5.0]), _f([10.0]), _f([0.0]), _f([5.0])) == 1
    assert sbm(_f([0.0]), _f([5.0]), _f([np.nextafter(np.float32(5), np.float32(9))]),
               _f([10.0])) == 0
    # a point inside, at either end of, and outside an interval
    for x, want in ((5.0, 1), (0.0, 1), (10.0, 1), (10.5, 0), (-0.5, 0)):
        assert sbm(_f([x]), _f([x]), _f([0.0]), _f([10.0])) == want, x
    # two equal points, and two different ones
    assert sbm(_f([3.0]), _f([3.0]), _f([3.0]), _f([3.0])) == 1
    assert sbm(_f([3.0]), _f([3.0]), _f([4.0]), _f([4.0])) == 0
    # boxes touching at a corner in 2-D and 3-D
    assert sbm(_f([[0, 0]]), _f([[1, 1]]), _f([[1, 1]]), _f([[2, 2]])) == 1
    assert sbm(_f([[0, 0, 0]]), _f([[1, 1, 1]]), _f([[1, 1, 1]]), _f([[2, 2, 2]])) == 1
    # zero width on the second axis only: a segment crossing a box
    assert sbm(_f([[0, 3]]), _f([[10, 3]]), _f([[1, 0]]), _f([[2, 9]])) == 1
    # chain: every neighbour touches, all at once
    lo = _f(np.arange(0, 10, 1)); hi = lo + 1
    k, per, pairs = oracle.sbm(lo, hi, lo, hi, closed=True)
    assert k == 10 + 2 * 9
    # signed zero and infinities
    nz = np.float32(-0.0)
    assert sbm(_f([-1.0]), _f([nz]), _f([0.0]), _f([1.0])) == 1
    inf = np.float32(np.inf)
    assert sbm(_f([inf]), _f([inf]), _f([0.0]), _f([inf])) == 1
    assert sbm(_f([-inf]), _f([-inf]), _f([-inf]), _f([0.0])) == 1


def test_closed_invalid_inputs_are_rejected(oracle):
    bad = [(_f([np.nan]), _f([1.0]), _f([0.0]), _f([1.0])),
           (_f([2.0]), _f([1.0]), _f([0.0]), _f([1.0]))]
    for args in bad:
        for fn in (oracle.sbm, oracle.bruteforce):
            with pytest.raises(O.OracleError):
                fn(*args, closed=True)
