"""GPU tests of resident simulations matched incrementally (ddm_resident_*):
every step's count against the matching oracle on the states replayed by
the CPU reference of the motion (tolerance 0: counts are integers), the
resident coordinates against that replay bit for bit, and the paths that
leave the slabs: movers that overflow their list or slab (repair by the full
call and a rebuild), boundary states that do not fit (full-match mode), d > 3,
empty regions, invalid input and misuse of the step protocol."""
import sys

import numpy as np
import pytest

from oracle import walk
from paper_1703_06680_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ddm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_06680_amd import ddm as D
    D.library()
    return D


def _dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def _sim(n, d, alpha, seed, sigma_scale=0.1):
    """n = m regions uniform on [0, 1e6)^d, side alpha * 1e6 / (2n)."""
    inst = W.uniform_instance(n, n, d, alpha, seed=seed)
    side = W.side_length(alpha, 2 * n)
    return inst, float(side), float(np.float32(sigma_scale) * side), 1000 + seed


def _run_and_check(ddm, oracle, inst, side, sigma, seed, steps):
    r = ddm.Resident(*_dev(inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi), side, sigma,
                     seed)
    for st, ul, uh, sl, sh in walk.walk(inst.upd_lo, inst.sub_lo, side, sigma, seed, steps):
        got = r.step(st)
        want, _, _ = oracle.sbm(ul, uh, sl, sh, pairs=False, per_update=False)
        assert got == want, (st, got, want)
    return r, (ul, uh, sl, sh)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("alpha", [1.0, 30.0])
def test_resident_counts_and_state_equal_oracle(ddm, oracle, d, alpha):
    inst, side, sigma, seed = _sim(12_000, d, alpha, seed=10 * d + int(alpha))
    _note(f"resident d={d} alpha={alpha} n=m={inst.n}")
    r, last = _run_and_check(ddm, oracle, inst, side, sigma, seed, steps=6)
    info = r.info()
    assert info["steps"] == 6 and info["full_mode"] == 0 and info["full_matches"] == 0
    assert info["buckets"] == (2 * inst.n + 1535) // 1536
    for dev, ref in zip(r.export(), last):
        assert np.array_equal(dev.cpu().numpy(), ref)
    r.close()


def test_resident_movers_cross_buckets(ddm, oracle):
    """A walk wide enough that hundreds of regions change bucket every step,
    all inserted into their new slabs (no repair)."""
    inst, side, _, seed = _sim(40_000, 2, 5.0, seed=31)
    sigma = 300.0  # buckets are about 19e3 wide
    _note("resident movers d=2 n=m=40000 sigma=300")
    r, last = _run_and_check(ddm, oracle, inst, side, sigma, seed, steps=5)
    info = r.info()
    assert info["movers"] > 100 and info["full_matches"] == 0 and info["rebuilds"] == 0
    for dev, ref in zip(r.export(), last):
        assert np.array_equal(dev.cpu().numpy(), ref)
    r.close()


def test_resident_overflowing_movers_are_repaired(ddm, oracle):
    """A walk of a third of the bucket width per step moves more regions than
    the mover list holds: the step is counted by the full call and the slabs
    are rebuilt; the second such step in a row turns the simulation to
    full-match mode.  With sigma far above the bucket width the regions left
    misplaced also overflow the boundary state, which turns it to full-match
    mode at once.  Counts and state stay exact throughout."""
    for n, d, sigma, rebuilt in ((20_000, 2, 1.0e4, True), (2_300, 1, 2.0e5, False)):
        inst, side, _, seed = _sim(n, d, 3.0, seed=40 + d)
        _note(f"resident overflow d={d} n=m={n} sigma={sigma}")
        r, last = _run_and_check(ddm, oracle, inst, side, sigma, seed, steps=4)
        info = r.info()
        assert info["full_matches"] >= 2 and info["full_mode"] == 1, info
        if rebuilt:
            assert info["rebuilds"] == 1, info
        for dev, ref in zip(r.export(), last):
            assert np.array_equal(dev.cpu().numpy(), ref)
        r.close()


def test_resident_boundary_state_overflow(ddm, oracle):
    """Regions so long that more than 512 are active at a bucket boundary:
    the first step is counted by the full call and the simulation stays in
    full-match mode, exactly."""
    inst, side, sigma, seed = _sim(6_000, 2, 600.0, seed=52)
    _note(f"resident long regions d=2 n=m=6000 side={side}")
    r, last = _run_and_check(ddm, oracle, inst, side, sigma, seed, steps=3)
    info = r.info()
    assert info["full_mode"] == 1 and info["full_matches"] == 3
    for dev, ref in zip(r.export(), last):
        assert np.array_equal(dev.cpu().numpy(), ref)
    r.close()


def test_resident_d5_and_empty(ddm, oracle):
    """d > 3 is matched by the full call at every step; no regions at all
    count 0."""
    inst, side, sigma, seed = _sim(3_000, 5, 2.0, seed=61)
    _note("resident d=5")
    r, _ = _run_and_check(ddm, oracle, inst, side, sigma, seed, steps=2)
    assert r.info()["full_mode"] == 1
    r.close()
    e = np.zeros((0, 2), np.float32)
    r0 = ddm.Resident(*_dev(e, e, e, e), 1.0, 0.1, 5)
    assert r0.step(1) == 0 and r0.step(2) == 0
    r0.close()


def test_resident_parked_empty_regions(ddm, oracle):
    """Regions far enough out that lo + side rounds back to lo are empty:
    they wait in the extra slab, match nothing, and keep moving."""
    inst, side, sigma, seed = _sim(5_000, 2, 4.0, seed=71)  # side 400
    for lo, hi in ((inst.upd_lo, inst.upd_hi), (inst.sub_lo, inst.sub_hi)):
        lo[:40, 0] += np.float32(3.0e10)  # spacing 2048 there: lo + 400 rounds to lo
        hi[:40, 0] = lo[:40, 0] + np.float32(side)
        assert np.all(hi[:40, 0] == lo[:40, 0])
    _note("resident parked empties d=2")
    r, last = _run_and_check(ddm, oracle, inst, side, sigma, seed, steps=4)
    assert r.info()["full_mode"] == 0
    for dev, ref in zip(r.export(), last):
        assert np.array_equal(dev.cpu().numpy(), ref)
    r.close()


def test_resident_invalid_input_and_protocol(ddm):
    inst, side, sigma, seed = _sim(2_000, 2, 1.0, seed=81)
    bad = inst.upd_lo.copy()
    bad[5, 1] = np.nan
    with pytest.raises(ddm.DDMError) as e:
        ddm.Resident(*_dev(bad, inst.upd_hi, inst.sub_lo, inst.sub_hi), side, sigma, seed)
    assert e.value.code == ddm.DDM_E_INVAL
    flipped = inst.sub_hi.copy()
    flipped[3, 0] = inst.sub_lo[3, 0] - 1.0
    with pytest.raises(ddm.DDMError) as e:
        ddm.Resident(*_dev(inst.upd_lo, inst.upd_hi, inst.sub_lo, flipped), side, sigma, seed)
    assert e.value.code == ddm.DDM_E_INVAL
    r = ddm.Resident(*_dev(inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi), side, sigma, seed)
    with pytest.raises(ddm.DDMError):
        r.finish()          # nothing pending
    with pytest.raises(ddm.DDMError):
        r.step_async(0)     # steps are numbered from 1
    r.step_async(1)
    with pytest.raises(ddm.DDMError):
        r.step_async(2)     # the pending step is not finished
    with pytest.raises(ddm.DDMError):
        r.export()
    r.finish()
    r.close()


def test_resident_full_size_against_oracle(ddm, oracle):
    """The benchmark's resident workload kind at full size (d = 2, n = m =
    5e6, alpha = 30 so that the counts are not trivially small): two steps,
    each count against the oracle on the C replay of the motion, and the
    final state against that replay bit for bit."""
    n, d, alpha = 5_000_000, 2, 30.0
    inst = W.uniform_instance(n, n, d, alpha, seed=11)
    side = float(W.side_length(alpha, 2 * n))
    sigma = float(np.float32(0.1) * np.float32(side))
    seed = 0x5EED
    _note(f"resident full size d={d} n=m={n} alpha={alpha}")
    r = ddm.Resident(*_dev(inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi), side, sigma, seed)
    for st, ul, uh, sl, sh in walk.walk_fast(inst.upd_lo, inst.sub_lo, side, sigma, seed, 2):
        got = r.step(st)
        want, _, _ = oracle.sbm(ul, uh, sl, sh, pairs=False, per_update=False)
        _note(f"step {st}: {got} pairs, oracle {want}")
        assert got == want
    info = r.info()
    assert info["full_matches"] == 0 and info["movers"] > 0
    for dev, ref in zip(r.export(), (ul, uh, sl, sh)):
        assert np.array_equal(dev.cpu().numpy(), ref)
    r.close()


def test_resident_retries_the_slabs(ddm, oracle):
    """2500 regions empty at creation overflow the slab of empty regions, so
    the simulation starts in full-match mode; the first step gives them their
    side back, and the retry after 64 full-match steps returns the simulation
    to the slabs.  Every count is exact throughout."""
    inst, side, sigma, seed = _sim(10_000, 2, 5.0, seed=95)
    inst.upd_hi[:2500, 1] = inst.upd_lo[:2500, 1]
    _note("resident retry d=2 n=m=10000, 2500 empty at creation")
    r = ddm.Resident(*_dev(inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi), side, sigma, seed)
    assert r.info()["full_mode"] == 1
    for st, ul, uh, sl, sh in walk.walk_fast(inst.upd_lo, inst.sub_lo, side, sigma, seed, 70):
        got = r.step(st)
        want, _, _ = oracle.sbm(ul, uh, sl, sh, pairs=False, per_update=False)
        assert got == want, st
        if st == 63:
            assert r.info()["full_mode"] == 1
    info = r.info()
    assert info["full_mode"] == 0 and info["rebuilds"] == 1 and info["full_matches"] == 64, info
    for dev, ref in zip(r.export(), (ul, uh, sl, sh)):
        assert np.array_equal(dev.cpu().numpy(), ref)
    r.close()
