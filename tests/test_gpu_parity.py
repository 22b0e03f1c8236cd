"""GPU parity: the HIP path (through the C interface) against the CPU oracle.

Every comparison is exact: counts, per-update counts and the lexicographically
ordered pair list must be identical element by element.  Inputs come from the
seeded generators shared with the oracle tests.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
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


def _dev(inst):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda()
            for a in (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)]


def _host(inst):
    return (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)


PATHS = ("auto", "global")


@pytest.fixture(autouse=True)
def _reset_path(ddm):
    ddm.set_path("auto")
    yield
    ddm.set_path("auto")


def check_all_modes(ddm, oracle, inst, pairs=True, expect_bucketed=None, closed=False):
    """Every output mode, on both implementations, equal to the oracle
    (closed boxes with ``closed``).  Returns the implementation that served
    the "auto" calls."""
    k_ref, per_ref, pairs_ref = oracle.sbm(*_host(inst), pairs=pairs, closed=closed)
    g = _dev(inst)
    served = None
    for path in PATHS:
        _note(f"{inst.name} n={inst.n} m={inst.m} d={inst.d} path={path} closed={closed}")
        ddm.set_path(path)
        k = ddm.match(*g, mode="count", closed=closed)
        assert k == k_ref, (inst.name, path, k, k_ref)
        if path == "auto":
            served = ddm.last_path()
        k1, per = ddm.match(*g, mode="per_update", closed=closed)
        assert k1 == k_ref, (inst.name, path)
        assert np.array_equal(per.cpu().numpy(), per_ref), (inst.name, path)
        if pairs:
            k2, pr, per2 = ddm.match(*g, mode="pairs", closed=closed)
            assert k2 == k_ref, (inst.name, path)
            assert np.array_equal(pr.cpu().numpy(), pairs_ref), (inst.name, path)
            assert np.array_equal(per2.cpu().numpy(), per_ref), (inst.name, path)
            k3, row_off, ids = ddm.match(*g, mode="csr", closed=closed)
            assert k3 == k_ref, (inst.name, path)
            want_off = np.concatenate([[0], np.cumsum(per_ref, dtype=np.int64)])
            assert np.array_equal(row_off.cpu().numpy(), want_off), (inst.name, path)
            assert np.array_equal(ids.cpu().numpy(), pairs_ref[:, 1]), (inst.name, path)
    ddm.set_path("auto")
    if expect_bucketed is None:
        expect_bucketed = inst.d <= 8 and inst.n + inst.m > 0
    if expect_bucketed:
        assert served == "bucketed", (inst.name, served)
    return served


def test_worked_example(ddm, oracle):
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ddm_example_fig.json")))
    arrs = [torch.tensor(g[k], dtype=torch.float32).cuda() for k in ("upd_lo", "upd_hi", "sub_lo", "sub_hi")]
    k, pairs, per = ddm.match(*arrs, mode="pairs")
    assert k == 4 and pairs.cpu().tolist() == g["expected_pairs"]
    assert per.cpu().tolist() == [2, 2]


def test_cfg1_full(ddm, oracle):
    check_all_modes(ddm, oracle, W.config_instance("cfg1"))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_tie_heavy_small(ddm, oracle, d):
    rng = np.random.default_rng(77 + d)
    for seed in range(40):
        n, m = int(rng.integers(0, 60)), int(rng.integers(0, 60))
        inst = W.tie_heavy(n, m, d, grid=int(rng.integers(2, 20)), max_len=int(rng.integers(0, 6)),
                           seed=seed)
        # tiny inputs with many empty boxes may legitimately have nothing to bucket
        check_all_modes(ddm, oracle, inst, expect_bucketed=False)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_tie_heavy_many_buckets(ddm, oracle, d):
    """Integer grid with heavy ties, large enough for thousands of buckets and
    long boundary-state lists."""
    inst = W.tie_heavy(30_000, 25_000, d, grid=4000, max_len=40, seed=11)
    check_all_modes(ddm, oracle, inst)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 9])
def test_random_float_boxes(ddm, oracle, d):
    for seed in range(6):
        check_all_modes(ddm, oracle, W.random_float_boxes(700, 900, d, seed=seed, extent=300.0),
                        expect_bucketed=d <= 8)


@pytest.mark.parametrize("d", [4, 6, 8])
def test_high_d_bucketed_with_many_matches(ddm, oracle, d):
    """d = 4 .. 8 on the bucketed path (pre-filter on axes 1 and 2, exact
    test on every axis), with boxes dense enough that thousands of pairs
    overlap on all d axes."""
    for seed in range(3):
        inst = W.random_float_boxes(2000, 2000, d, seed=seed, extent=40.0)
        check_all_modes(ddm, oracle, inst, expect_bucketed=True)


def test_high_d_full_counts(ddm, oracle):
    """d = 5, n = m = 5e6, alpha = 30: total and per-update counts on the
    bucketed path against the oracle."""
    inst = W.uniform_instance(5_000_000, 5_000_000, 5, 30.0, seed=21)
    _note(f"{inst.name}")
    g = _dev(inst)
    k_ref, per_ref, _ = oracle.sbm(*_host(inst), pairs=False)
    k, per = ddm.match(*g, mode="per_update")
    assert ddm.last_path() == "bucketed"
    assert k == k_ref
    assert np.array_equal(per.cpu().numpy(), per_ref)


@pytest.mark.parametrize("d,alpha", [(1, 100.0), (2, 1.0), (3, 100.0)])
def test_multi_tile_with_ragged_tail(ddm, oracle, d, alpha):
    # sizes that span many sort tiles and sweep blocks, none a multiple of a tile
    check_all_modes(ddm, oracle, W.uniform_instance(20_011, 17_389, d, alpha, seed=4))


@pytest.mark.parametrize("alpha", [0.01, 1.0, 100.0])
def test_cfg2_full(ddm, oracle, alpha):
    """d=2, n = m = 5e5 at every alpha of the configuration."""
    check_all_modes(ddm, oracle, W.config_instance("cfg2", alpha))


@pytest.mark.parametrize("alpha", [1.0, 10.0, 100.0])
def test_cfg3_full_counts(ddm, oracle, alpha):
    """d=3, n = m = 5e6: exact total and per-update counts on both paths."""
    inst = W.config_instance("cfg3", alpha)
    g = _dev(inst)
    k_ref, per_ref, _ = oracle.sbm(*_host(inst), pairs=False)
    for path in PATHS:
        _note(f"{inst.name} path={path}")
        ddm.set_path(path)
        k, per = ddm.match(*g, mode="per_update")
        assert k == k_ref
        assert np.array_equal(per.cpu().numpy(), per_ref)
        if path == "auto":
            assert ddm.last_path() == "bucketed"


def test_more_buckets_than_the_pair_scatter_holds(ddm, oracle):
    """n = m = 5.5e6 (7162 buckets, beyond the 6656 the pairing scatter keeps
    in LDS): the single-store scatter, per-update counts against the 1-D
    closed form, and pairs of a sample of updates against the oracle's."""
    from oracle import oracle as O
    inst = W.uniform_instance(5_500_000, 5_500_000, 1, 20.0, seed=8)
    _note(f"{inst.name} beyond the pairing scatter")
    g = _dev(inst)
    ddm.set_path("bucketed")
    k, per = ddm.match(*g, mode="per_update")
    want = O.closed_form_1d(*_host(inst))
    assert np.array_equal(per.cpu().numpy().astype(np.int64), want)
    assert k == int(want.sum())
    # the sampled updates' rows of the pair list against the oracle's
    k2, pairs, _ = ddm.match(*g, mode="pairs")
    assert k2 == k
    pairs = pairs.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(want)])
    rows = np.random.default_rng(3).choice(inst.n, size=200, replace=False)
    sub = (inst.upd_lo[rows], inst.upd_hi[rows], inst.sub_lo, inst.sub_hi)
    _, _, ref = oracle.sbm(*sub)
    for i, r in enumerate(rows):
        got = pairs[off[r]:off[r + 1], 1]
        assert np.array_equal(got, ref[ref[:, 0] == i, 1]), r


@pytest.mark.parametrize("d", [2, 3, 5])
@pytest.mark.parametrize("closed", [False, True])
def test_grid_cells(ddm, oracle, d, closed):
    """Inputs whose walks in swept-axis slabs would be long (alpha = 40,
    about 20 entries), so the plan cuts the slabs into rows by axis 1: every
    mode on both paths, on float boxes and on an integer lattice whose
    coordinates fall on cell boundaries (touching and point boxes)."""
    inst = W.uniform_instance(30_000, 25_000, d, 40.0, seed=11 + d)
    check_all_modes(ddm, oracle, inst, closed=closed)
    ties = W.tie_heavy(30_000, 30_000, d, grid=300, max_len=8, seed=d)
    check_all_modes(ddm, oracle, ties, closed=closed)


def test_grid_rows_with_long_axis1_boxes(ddm, oracle):
    """Grid rows with boxes that reach many later rows of their column
    (copies as records) beside small ones, and boxes that also cross into
    later columns (boundary-state copies in several rows)."""
    rng = np.random.default_rng(5)
    n = m = 30_000
    lo = (rng.random((n + m, 3)) * 1000.0).astype(np.float32)
    side = np.full((n + m, 3), 10.0, dtype=np.float32)
    long1 = rng.random(n + m) < 0.02
    side[long1, 1] = 400.0
    long0 = rng.random(n + m) < 0.01
    side[long0, 0] = 150.0
    hi = (lo + side).astype(np.float32)
    inst = W.Instance(lo[:n], hi[:n], lo[n:], hi[n:], float("nan"), "long_axis1_rows")
    check_all_modes(ddm, oracle, inst)


@pytest.mark.parametrize("alpha", [1.0, 100.0])
def test_correlated_d3_stress(ddm, oracle, alpha):
    """Many true 3-D matches, so per-update counts and pairs are exercised."""
    inst = W.correlated_d3(400_000, alpha, seed=2)
    check_all_modes(ddm, oracle, inst)


def test_swept_axis_choice(ddm, oracle):
    """Boxes 100 times longer on axis 0 than on axes 1 and 2: the plan sweeps
    another axis; every forced axis gives the same result, equal to the
    oracle in every output mode."""
    inst = W.anisotropic_boxes(60_000, 50_000, 3, 30.0, seed=5)
    try:
        for axis in (None, 0, 1, 2):
            ddm.set_sweep_axis(axis)
            check_all_modes(ddm, oracle, inst, expect_bucketed=True)
        ddm.set_sweep_axis(None)
        closed = W.anisotropic_boxes(40_000, 45_000, 2, 20.0, seed=6)
        check_all_modes(ddm, oracle, closed, closed=True, expect_bucketed=True)
        ddm.set_sweep_axis(7)  # beyond d: axis 0
        check_all_modes(ddm, oracle, closed, expect_bucketed=True)
        with pytest.raises(ddm.DDMError):
            ddm.set_sweep_axis(-2)
    finally:
        ddm.set_sweep_axis(None)


@pytest.mark.parametrize("kind", ["loguniform", "clustered"])
def test_skewed_inputs_split_buckets(ddm, oracle, kind):
    """Lower corners spread over six decades (sides proportional to them) or
    packed into 16 normal clusters: buckets of the sampled linear map hold
    far more records than a sweep workgroup can; their exact totals split
    them and the call stays on the bucketed path.  Every output mode on both
    paths equal to the oracle, half-open and closed."""
    make = W.loguniform_boxes if kind == "loguniform" else W.clustered_boxes
    for d in (1, 2, 3):
        inst = make(100_000, 90_000, d, 40.0, seed=d)
        check_all_modes(ddm, oracle, inst, expect_bucketed=True)
    inst = make(60_000, 70_000, 2, 40.0, seed=9)
    check_all_modes(ddm, oracle, inst, closed=True, expect_bucketed=True)


def test_other_axes_over_many_magnitudes(ddm, oracle):
    """Axes 1 and 2 spread over six decades on both sides of zero (a few
    boxes across it): the plan quantises them on the encoded coordinate.
    Every output mode on both paths equal to the oracle, half-open and
    closed."""
    for d in (2, 3):
        inst = W.signed_logscale_boxes(100_000, 90_000, d, 40.0, seed=d, other_alpha=2000.0)
        check_all_modes(ddm, oracle, inst, expect_bucketed=True)
    inst = W.signed_logscale_boxes(60_000, 70_000, 3, 40.0, seed=9, other_alpha=3000.0)
    check_all_modes(ddm, oracle, inst, closed=True, expect_bucketed=True)


def test_heavy_buckets_grid_and_closed(ddm, oracle):
    """Buckets whose quantised pre-filter passes more pairs than the sweep's
    queue holds are listed and swept again with the exact bounds of axes 1
    and 2 staged on chip (per-update counts from the updates' side): the
    correlated boxes as closed boxes, and dense d = 2 boxes on a grid of
    cells (thousands of true matches per cell, counted in one row)."""
    inst = W.correlated_d3(150_000, 100.0, seed=4)
    check_all_modes(ddm, oracle, inst, closed=True, expect_bucketed=True)
    dense = W.uniform_instance(200_000, 200_000, 2, 2000.0, seed=6)
    check_all_modes(ddm, oracle, dense, expect_bucketed=True)


# ------------------------------------------------------------- edge cases

def _t(a, d=1):
    return torch.tensor(np.asarray(a, dtype=np.float32).reshape(-1, d)).cuda()


def test_empty_sets(ddm):
    _note("empty sets")
    z = torch.zeros((0, 2), dtype=torch.float32, device="cuda")
    one = torch.ones((5, 2), dtype=torch.float32, device="cuda")
    assert ddm.match(z, z, one * 0, one) == 0
    assert ddm.match(one * 0, one, z, z) == 0
    k, per = ddm.match(one * 0, one, z, z, mode="per_update")
    assert k == 0 and per.cpu().tolist() == [0] * 5
    k, pairs, _ = ddm.match(z, z, z, z, mode="pairs")
    assert k == 0 and pairs.shape == (0, 2)


def test_all_identical_gives_n_times_m(ddm):
    _note("all identical")
    lo = torch.full((300, 3), 2.0, device="cuda")
    hi = torch.full((300, 3), 9.0, device="cuda")
    slo = torch.full((200, 3), 2.0, device="cuda")
    shi = torch.full((200, 3), 9.0, device="cuda")
    k, pairs, per = ddm.match(lo, hi, slo, shi, mode="pairs")
    assert k == 60_000
    exp = np.stack(np.meshgrid(np.arange(300), np.arange(200), indexing="ij"), -1).reshape(-1, 2)
    assert np.array_equal(pairs.cpu().numpy(), exp)
    assert per.cpu().tolist() == [200] * 300


def test_touching_nested_signed_zero_infinity(ddm):
    _note("touching / nested / signed zero / inf")
    assert ddm.match(_t([0, 2, 4]), _t([1, 3, 5]), _t([1, 3, 5]), _t([2, 4, 6])) == 0
    assert ddm.match(_t([2.0]), _t([3.0]), _t([0.0]), _t([10.0])) == 1
    assert ddm.match(_t([-0.0]), _t([1.0]), _t([0.0]), _t([1.0])) == 1
    assert ddm.match(_t([-1.0]), _t([-0.0]), _t([0.0]), _t([1.0])) == 0
    inf = float("inf")
    assert ddm.match(_t([-inf]), _t([inf]), _t([0.0]), _t([1.0])) == 1
    assert ddm.match(_t([inf]), _t([inf]), _t([0.0]), _t([inf])) == 0
    assert ddm.match(_t([5.0]), _t([5.0]), _t([0.0]), _t([10.0])) == 0


def test_invalid_input_is_reported(ddm):
    _note("invalid input")
    nan = float("nan")
    for args in ((_t([nan]), _t([1.0]), _t([0.0]), _t([1.0])),
                 (_t([2.0]), _t([1.0]), _t([0.0]), _t([1.0])),
                 (_t([[0, 2]], 2), _t([[1, 1]], 2), _t([[0, 0]], 2), _t([[1, 1]], 2))):
        with pytest.raises(ddm.DDMError) as e:
            ddm.match(*args)
        assert e.value.code == ddm.DDM_E_INVAL


def test_copy_probe_copies_and_times(ddm):
    """The library's bandwidth yardstick copies its input exactly and
    reports a positive time and a plausible rate."""
    _note("copy probe")
    src = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    ms = ddm.ctypes.c_double(0.0)
    rc = ddm.library().ddm_copy_probe(ddm.ctypes.c_void_p(dst.data_ptr()),
                                      ddm.ctypes.c_void_p(src.data_ptr()), src.numel() * 4, 3,
                                      ddm.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                      ddm.ctypes.byref(ms))
    torch.cuda.synchronize()
    assert rc == 0 and ms.value > 0
    assert torch.equal(dst, src)
    c = ddm.copy_probe(64 << 20, reps=3)
    assert c["bytes_moved"] == 128 << 20 and 100 < c["gb_per_s"] < 8000


def test_capacity_retry(ddm, oracle):
    _note("capacity retry")
    inst = W.tie_heavy(50, 50, 2, grid=5, seed=1)
    g = _dev(inst)
    k_ref, _, pairs_ref = oracle.sbm(*_host(inst))
    assert k_ref > 10
    with pytest.raises(ddm.DDMError) as e:
        ddm.match(*g, mode="pairs", pair_capacity=k_ref - 1)
    assert e.value.code == ddm.DDM_E_CAPACITY
    k, pairs, _ = ddm.match(*g, mode="pairs", pair_capacity=k_ref)
    assert k == k_ref and np.array_equal(pairs.cpu().numpy(), pairs_ref)


def test_deterministic_and_permutation_invariant(ddm, oracle):
    _note("determinism / permutation")
    inst = W.correlated_d3(50_000, 100.0, seed=5)
    g = _dev(inst)
    k1, p1, c1 = ddm.match(*g, mode="pairs")
    k2, p2, c2 = ddm.match(*g, mode="pairs")
    assert k1 == k2 and torch.equal(p1, p2) and torch.equal(c1, c2)
    rng = np.random.default_rng(0)
    pu, ps = rng.permutation(inst.n), rng.permutation(inst.m)
    gp = [g[0][pu], g[1][pu], g[2][ps], g[3][ps]]
    k3, p3, _ = ddm.match(*gp, mode="pairs")
    assert k3 == k1
    mapped = np.stack([pu[p3[:, 0].cpu().numpy()], ps[p3[:, 1].cpu().numpy()]], 1)
    mapped = mapped[np.lexsort((mapped[:, 1], mapped[:, 0]))]
    assert np.array_equal(mapped, p1.cpu().numpy())


def test_role_swap_transposes(ddm):
    _note("role swap")
    inst = W.random_float_boxes(2000, 1500, 2, seed=3, extent=200.0)
    g = _dev(inst)
    k, p, _ = ddm.match(*g, mode="pairs")
    k2, p2, _ = ddm.match(g[2], g[3], g[0], g[1], mode="pairs")
    assert k == k2
    t = p2.cpu().numpy()[:, ::-1]
    t = t[np.lexsort((t[:, 1], t[:, 0]))]
    assert np.array_equal(t, p.cpu().numpy())


def test_overflowing_bucket_falls_back(ddm, oracle):
    """3000 identical boxes per side land in one bucket, larger than a
    workgroup can hold: "auto" must fall back to the device-wide path, and
    forcing the bucketed path must refuse rather than answer."""
    _note("overflowing bucket")
    lo = np.full((3000, 2), 1.0, np.float32)
    hi = np.full((3000, 2), 4.0, np.float32)
    g = [torch.from_numpy(a).cuda() for a in (lo, hi, lo.copy(), hi.copy())]
    k, per = ddm.match(*g, mode="per_update")
    assert k == 9_000_000 and ddm.last_path() == "global"
    assert per.cpu().tolist() == [3000] * 3000
    ddm.set_path("bucketed")
    with pytest.raises(ddm.DDMError) as e:
        ddm.match(*g, mode="count")
    assert e.value.code == ddm.DDM_E_UNSUPPORTED


def test_skewed_distribution(ddm, oracle):
    """Lower corners spread over six orders of magnitude (log-uniform): the
    linear bucket map is badly balanced, and the answer must not change."""
    rng = np.random.default_rng(3)
    for d in (1, 3):
        n = 60_000
        lo = np.exp(rng.uniform(0, np.log(1e6), size=(2 * n, d))).astype(np.float32)
        side = np.exp(rng.uniform(np.log(0.5), np.log(50.0), size=(2 * n, d))).astype(np.float32)
        hi = (lo + side).astype(np.float32)
        inst = W.Instance(lo[:n], hi[:n], lo[n:], hi[n:], float("nan"), f"loguniform_d{d}")
        check_all_modes(ddm, oracle, inst, expect_bucketed=False)


def test_boundary_state_beyond_capacity_falls_back(ddm, oracle):
    """2000 subscriptions reaching from a random point to past the end of
    the swept axis and over the whole of axis 1 (d = 2, n = m = 5e5): copied
    into the boundary state of every later bucket they would need about
    6.5e5 entries, more than the buffer's 5.04e5.  The count pass stops
    counting them once the total passes the capacity, the scatter and the
    sweep stand down, and the call is answered by the device-wide path with
    the oracle's counts.  With 1000 such subscriptions (about 3.3e5 copies)
    the bucketed path holds them."""
    for long_subs, path in ((2000, "global"), (1000, "bucketed")):
        inst = W.uniform_instance(500_000, 500_000, 2, 1.0, seed=21)
        rng = np.random.default_rng(22)
        sel = rng.choice(inst.m, size=long_subs, replace=False)
        inst.sub_hi[sel, 0] = 2.0e6
        inst.sub_lo[sel, 1] = -1.0
        inst.sub_hi[sel, 1] = 2.0e6
        k_ref, per_ref, _ = oracle.sbm(*_host(inst), pairs=False)
        assert k_ref >= long_subs * 100_000
        g = _dev(inst)
        _note(f"{long_subs} long subscriptions, per_update")
        k, per = ddm.match(*g, mode="per_update")
        assert (ddm.last_path(), k) == (path, k_ref)
        assert np.array_equal(per.cpu().numpy(), per_ref)
        _note(f"{long_subs} long subscriptions, count (graph replay)")
        for _ in range(3):  # eager, captured, replayed
            assert ddm.match(*g, mode="count") == k_ref
            assert ddm.last_path() == path


@pytest.mark.parametrize("mode", ["count", "per_update"])
def test_repeated_call_replays_graph(ddm, oracle, mode):
    """Identical repeated calls are captured once and replayed: every replay
    reads the current contents of the same buffers, including contents that
    overflow a bucket (replay falls back to the device-wide path)."""
    n, m, d = 20_000, 18_000, 3
    g = [torch.empty((k, d), dtype=torch.float32, device="cuda") for k in (n, n, m, m)]
    ws = torch.empty(ddm.workspace_bytes(n, m, d, mode), dtype=torch.uint8, device="cuda")
    per = torch.empty(n, dtype=torch.int32, device="cuda")
    cases = [W.uniform_instance(n, m, d, 50.0, seed=s) for s in range(3)]
    lo = np.zeros((n, d), np.float32)
    hi = np.ones((n, d), np.float32)
    cases.append(W.Instance(lo, hi, lo[:m].copy(), hi[:m].copy(), float("nan"), "identical"))
    cases += [W.correlated_d3(n, 20.0, seed=5), W.uniform_instance(n, m, d, 5.0, seed=9)]
    cases[4] = W.Instance(cases[4].upd_lo, cases[4].upd_hi, cases[4].sub_lo[:m], cases[4].sub_hi[:m],
                          cases[4].alpha, "correlated")
    for rep, inst in enumerate(cases + cases[:2]):
        for dst, src in zip(g, (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)):
            dst.copy_(torch.from_numpy(np.ascontiguousarray(src)))
        k_ref, per_ref, _ = oracle.sbm(inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi,
                                       pairs=False)
        _note(f"replay {rep} {inst.name} mode={mode}")
        k = ddm.match_into(*g, mode=mode, workspace=ws, per_update=per if mode == "per_update" else None)
        assert k == k_ref, (rep, inst.name)
        if mode == "per_update":
            assert np.array_equal(per.cpu().numpy(), per_ref), (rep, inst.name)


@pytest.mark.parametrize("inst_fn", [
    lambda: W.uniform_instance(300_000, 250_000, 3, 30.0, seed=4),
    lambda: W.tie_heavy(20_000, 15_000, 2, grid=300, max_len=12, seed=6),
    lambda: W.random_float_boxes(5000, 4000, 4, seed=8, extent=300.0),
])
def test_dim_counts_equal_closed_form(ddm, inst_fn):
    """K_1D of every axis equals the oracle's closed form summed over updates."""
    inst = inst_fn()
    g = _dev(inst)
    got = ddm.dim_counts(*g)
    want = [int(O.closed_form_1d(*_host(inst), axis=k).sum()) for k in range(inst.d)]
    _note(f"dim counts {inst.name}: {got}")
    assert got == want


# ------------------------------------------------------- closed intervals

@pytest.mark.parametrize("d", [1, 2, 3])
def test_closed_tie_heavy_small(ddm, oracle, d):
    rng = np.random.default_rng(177 + d)
    for seed in range(30):
        n, m = int(rng.integers(0, 60)), int(rng.integers(0, 60))
        inst = W.tie_heavy(n, m, d, grid=int(rng.integers(2, 20)), max_len=int(rng.integers(0, 6)),
                           seed=seed)
        check_all_modes(ddm, oracle, inst, expect_bucketed=inst.n + inst.m > 0, closed=True)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_closed_tie_heavy_many_buckets(ddm, oracle, d):
    """Points and touching intervals everywhere, thousands of buckets."""
    inst = W.tie_heavy(30_000, 25_000, d, grid=4000, max_len=40, seed=12)
    check_all_modes(ddm, oracle, inst, closed=True)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 9])
def test_closed_random_float_boxes(ddm, oracle, d):
    for seed in range(4):
        inst = W.random_float_boxes(700, 900, d, seed=seed, extent=300.0)
        check_all_modes(ddm, oracle, inst, expect_bucketed=d <= 8, closed=True)


def test_closed_infinite_and_zero_bounds(ddm, oracle):
    """Closed boxes reaching +-inf (enc(+inf) + 1 must not wrap) and points at
    signed zero."""
    rng = np.random.default_rng(5)
    inst = W.tie_heavy(3000, 3000, 2, grid=50, max_len=3, seed=5)
    ul, uh, sl, sh = (a.copy() for a in _host(inst))
    inf = np.float32(np.inf)
    for lo, hi in ((ul, uh), (sl, sh)):
        rows = rng.choice(lo.shape[0], 200, replace=False)
        hi[rows[:100], 0] = inf
        lo[rows[100:150], 0] = -inf
        lo[rows[150:], 1] = -0.0
        hi[rows[150:], 1] = 0.0
    check_all_modes(ddm, oracle, W.Instance(ul, uh, sl, sh, float("nan"), "closed_inf"),
                    closed=True)


@pytest.mark.parametrize("d,alpha", [(2, 1.0), (2, 100.0), (3, 100.0)])
def test_closed_paper_workload(ddm, oracle, d, alpha):
    inst = W.uniform_instance(200_000, 200_000, d, alpha, seed=21)
    check_all_modes(ddm, oracle, inst, pairs=d == 2, closed=True)


def test_closed_full_size_equals_half_open_next_float(ddm):
    """At the d = 3, n = m = 5e6 size: closed [lo, hi] matches exactly as
    half-open [lo, nextafter(hi)), per update."""
    inst = W.uniform_instance(5_000_000, 5_000_000, 3, 100.0, seed=0)
    g = _dev(inst)
    up = [torch.nextafter(t, torch.tensor(float("inf"), device=t.device)) for t in (g[1], g[3])]
    _note("closed vs next-float half-open, d=3 n=m=5e6")
    kc, pc = ddm.match(*g, mode="per_update", closed=True)
    kh, ph = ddm.match(g[0], up[0], g[2], up[1], mode="per_update")
    assert kc == kh and torch.equal(pc, ph)


# ------------------------------------------------------------ CSR output

def test_csr_capacity_and_empty_cases(ddm, oracle):
    """K above the capacity: DDM_E_CAPACITY, the count set and the row
    offsets complete; no pairs, no updates, no subscriptions: empty rows."""
    import ctypes
    inst = W.tie_heavy(3000, 2000, 2, grid=200, max_len=8, seed=3)
    k_ref, per_ref, pairs_ref = oracle.sbm(*_host(inst))
    assert k_ref > 10
    g = _dev(inst)
    lib = ddm.library()
    n, m, d = inst.n, inst.m, inst.d
    cap = k_ref - 1
    ws = torch.empty(ddm.workspace_bytes(n, m, d, "pairs", cap), dtype=torch.uint8, device="cuda")
    row_off = torch.full((n + 1,), -7, dtype=torch.int64, device="cuda")
    ids = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    cnt = ctypes.c_uint64(0)
    for path in PATHS:
        ddm.set_path(path)
        row_off.fill_(-7)
        rc = lib.ddm_match_csr(*[ctypes.c_void_p(t.data_ptr()) for t in g[:2]], n,
                               *[ctypes.c_void_p(t.data_ptr()) for t in g[2:]], m, d, 0,
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), None, ctypes.byref(cnt),
                               ctypes.c_void_p(row_off.data_ptr()), ctypes.c_void_p(ids.data_ptr()),
                               cap)
        assert rc == ddm.DDM_E_CAPACITY and cnt.value == k_ref, (path, rc)
        want_off = np.concatenate([[0], np.cumsum(per_ref, dtype=np.int64)])
        assert np.array_equal(row_off.cpu().numpy(), want_off), path
        assert bool((ids == -7).all()), path
    ddm.set_path("auto")
    # a retry with the reported size succeeds
    k, ro, got = ddm.match(*g, mode="csr", pair_capacity=int(cnt.value))
    assert k == k_ref and np.array_equal(got.cpu().numpy(), pairs_ref[:, 1])
    # no pairs at all / no updates / no subscriptions
    far = [t + 1e5 for t in g[2:]]
    k, ro, got = ddm.match(g[0], g[1], far[0], far[1], mode="csr")
    assert k == 0 and not bool(ro.any()) and ro.numel() == n + 1 and got.numel() == 0
    z = torch.zeros((0, d), dtype=torch.float32, device="cuda")
    k, ro, got = ddm.match(z, z, g[2], g[3], mode="csr")
    assert k == 0 and ro.cpu().tolist() == [0]
    k, ro, got = ddm.match(g[0], g[1], z, z, mode="csr")
    assert k == 0 and ro.numel() == n + 1 and not bool(ro.any())
    # bad flags are rejected before any launch
    rc = lib.ddm_match_csr(*[ctypes.c_void_p(t.data_ptr()) for t in g[:2]], n,
                           *[ctypes.c_void_p(t.data_ptr()) for t in g[2:]], m, d, 1,
                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), None, ctypes.byref(cnt),
                           ctypes.c_void_p(row_off.data_ptr()), ctypes.c_void_p(ids.data_ptr()), cap)
    assert rc == ddm.DDM_E_INVAL


@pytest.mark.parametrize("rows", [(2048, 10, 1), (3000, 2048, 2049, 10)])
def test_pairs_rows_at_and_beyond_the_row_sort_limit(ddm, oracle, rows):
    """Rows of up to 2048 pairs are ordered one by one; a longer row sends
    the whole call to the device-wide sort.  Both must give the same,
    oracle-equal pair lists and CSR rows."""
    m = 3000
    slo = np.arange(m, dtype=np.float32).reshape(-1, 1)
    shi = slo + np.float32(0.5)
    ulo = np.zeros((len(rows), 1), np.float32)
    uhi = np.array([[r - 0.25] for r in rows], np.float32)  # row r covers subs 0 .. r-1
    inst = W.Instance(ulo, uhi, slo, shi, float("nan"), f"rows{rows}")
    k_ref, per_ref, _ = oracle.sbm(*_host(inst))
    assert per_ref.tolist() == list(rows)
    check_all_modes(ddm, oracle, inst, expect_bucketed=False)


def test_d1_rows_boundary_state_beyond_lds(ddm, oracle):
    """d = 1 pairs where some buckets carry more boundary-state subscriptions
    than the row emission holds in LDS, so the call falls back to emission
    pair by pair, while every row is short: 3000 long subscriptions on
    [0, 2000) that meet no update, and 20000 short updates on [2000, 12000)
    each with one subscription on top of it."""
    rng = np.random.default_rng(9)
    long_lo = (rng.random(3000) * 1000.0).astype(np.float32)
    long_hi = (long_lo + np.float32(1000.0)).astype(np.float32)
    u_lo = (2000.0 + rng.random(20000) * 10000.0).astype(np.float32)
    u_hi = (u_lo + np.float32(0.001)).astype(np.float32)
    slo = np.concatenate([long_lo, u_lo]).reshape(-1, 1)
    shi = np.concatenate([long_hi, u_hi]).reshape(-1, 1)
    inst = W.Instance(u_lo.reshape(-1, 1), u_hi.reshape(-1, 1), slo, shi, float("nan"),
                      "d1_wide_boundary_state")
    assert oracle.sbm(*_host(inst), pairs=False)[0] >= 20000
    check_all_modes(ddm, oracle, inst)
