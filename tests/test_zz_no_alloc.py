"""ddm_match_noalloc (the entry point that allocates nothing: its workspace
is the library's static device array) against ddm_match on the same inputs:
every output equal, element by element, on two calls in a row, the second
with a smaller input, in every output mode, on both implementation paths;
and sizes beyond the array refused on the device as on the host."""
import sys

import numpy as np
import pytest

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
    D.set_path("auto")
    return D


def _dev(inst):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda()
            for a in (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)]


def _both(ddm, g, mode, closed=False, cap=0):
    """(count, per-update, pairs) from ddm_match and from ddm_match_noalloc."""
    n = g[0].shape[0]
    out = []
    for which in ("match", "noalloc"):
        per = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        pairs = torch.full((cap, 2), -7, dtype=torch.int32, device="cuda") if mode == "pairs" else None
        if which == "match":
            ws = torch.empty(ddm.workspace_bytes(n, g[2].shape[0], g[0].shape[1], mode, cap, closed),
                             dtype=torch.uint8, device="cuda")
            k = ddm.match_into(*g, mode, ws, per if mode != "count" else None, pairs,
                               closed=closed)
        else:
            k = ddm.match_noalloc_into(*g, mode, per if mode != "count" else None, pairs,
                                       closed=closed)
        torch.cuda.synchronize()
        out.append((k, per.cpu().numpy(), pairs[:k].cpu().numpy() if pairs is not None else None))
    return out


CASES = [
    # (d, large n, small n, alpha)
    (1, 600_000, 40_000, 1.0),
    (2, 450_000, 30_000, 60.0),
    (3, 350_000, 25_000, 90.0),
]


@pytest.mark.parametrize("d,n_big,n_small,alpha", CASES)
@pytest.mark.parametrize("mode", ["count", "per_update", "pairs"])
def test_noalloc_equals_match_two_calls(ddm, d, n_big, n_small, alpha, mode):
    for call, n in enumerate((n_big, n_small)):
        inst = W.uniform_instance(n, n + 17, d, alpha, seed=40 + call)
        g = _dev(inst)
        cap = 0
        if mode == "pairs":
            cap = ddm.match(*g, mode="count") + 5
        _note(f"noalloc d={d} n={n} alpha={alpha} mode={mode} call={call}")
        (k0, p0, q0), (k1, p1, q1) = _both(ddm, g, mode, cap=cap)
        assert ddm.last_path() == "bucketed"
        assert k1 == k0
        if mode != "count":
            assert np.array_equal(p1, p0)
        if mode == "pairs":
            assert np.array_equal(q1, q0)
        if d <= 2:
            assert k0 > 0  # not a comparison of empty results


def test_noalloc_device_wide_path_and_closed_boxes(ddm):
    """Tie-heavy integer grids: closed boxes on the bucketed path, then the
    device-wide path (forced), a larger and then a smaller input."""
    try:
        for call, n in enumerate((200_000, 9_000)):
            t = W.tie_heavy(n, n - 11, 2, grid=2000, max_len=6, seed=70 + call)
            g = _dev(t)
            cap = ddm.match(*g, mode="count", closed=True) + 1
            _note(f"noalloc closed tie-heavy n={n} call={call}")
            (k0, p0, q0), (k1, p1, q1) = _both(ddm, g, "pairs", closed=True, cap=cap)
            assert k1 == k0 > 0 and np.array_equal(p1, p0) and np.array_equal(q1, q0)
            ddm.set_path("global")
            _note(f"noalloc global path n={n} call={call}")
            (k0, p0, _), (k1, p1, _) = _both(ddm, g, "per_update")
            assert ddm.last_path() == "global"
            assert k1 == k0 > 0 and np.array_equal(p1, p0)
            ddm.set_path("auto")
    finally:
        ddm.set_path("auto")


def test_noalloc_refuses_beyond_its_array_and_still_works_after(ddm):
    big = W.uniform_instance(1_200_000, 1_200_000, 2, 1.0, seed=3)
    g = _dev(big)
    _note("noalloc oversize request")
    with pytest.raises(ddm.DDMError) as e:
        ddm.match_noalloc_into(*g, "count")
    assert e.value.code == ddm.DDM_E_SCRATCH
    small = W.uniform_instance(5_000, 4_000, 2, 40.0, seed=4)
    gs = _dev(small)
    (k0, _, _), (k1, _, _) = _both(ddm, gs, "count")
    assert k1 == k0
