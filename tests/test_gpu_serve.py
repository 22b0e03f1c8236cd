"""GPU tests of the serving runtime: the device random walk against its CPU
reference bit for bit, served counts against the matching oracle on the
replayed states, every request's result identical alone and in the mix
(tolerance 0: counts are integers), admission under a tight HBM budget, and
the plain per-request policy."""
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


def _small_sims(count=6, seed=3):
    return W.serving_sims(count, d=2, seed=seed, lo=1_500, hi=20_000)


def _upload(inst):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda()
            for a in (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)]


def _expected_counts(oracle, inst, side, sigma, seed, steps):
    out = {}
    for st, ul, uh, sl, sh in walk.walk(inst.upd_lo, inst.sub_lo, side, sigma, seed, steps):
        k, _, _ = oracle.sbm(ul, uh, sl, sh, pairs=False, per_update=False)
        out[st] = k
    return out


def test_sim_step_matches_reference(ddm):
    inst, side, sigma, seed = _small_sims(1, seed=9)[0]
    g = _upload(inst)
    for st in range(1, 5):
        ddm.sim_step(*g, side, sigma, seed, st)
    torch.cuda.synchronize()
    *_, (st, ul, uh, sl, sh) = list(walk.walk(inst.upd_lo, inst.sub_lo, side, sigma, seed, 4))
    for dev, ref in zip(g, (ul, uh, sl, sh)):
        assert np.array_equal(dev.cpu().numpy(), ref)


def _server(ddm, sims, policy="batched", arena=1 << 30, slots=4, max_batch=8):
    sv = ddm.Server(arena, policy=policy, slots=slots, max_batch=max_batch)
    states = []
    for inst, side, sigma, seed in sims:
        g = _upload(inst)
        sv.add_sim(*g, side, sigma, seed)
        states.append(g)
    return sv, states


@pytest.mark.parametrize("policy", ["batched", "plain", "incremental"])
def test_served_counts_alone_equal_mix_equal_oracle(ddm, oracle, policy):
    sims = _small_sims(6)
    per_sim = 4
    expected = [_expected_counts(oracle, *s, per_sim) for s in sims]
    # in the mix: Poisson arrivals fast enough that requests overlap
    ids, arr = W.poisson_arrivals(6 * per_sim, qps=20000.0, seed=1, sims=6)
    # every simulation gets exactly per_sim requests
    ids = np.repeat(np.arange(6, dtype=np.int32), per_sim)
    np.random.default_rng(2).shuffle(ids)
    _note(f"serve mix policy={policy} requests={ids.size}")
    sv, states = _server(ddm, sims, policy)
    counts, steps, lat, stats = sv.run(ids, arr)
    assert np.all(lat >= 0) and stats["launches"] >= 1
    for i in range(ids.size):
        assert int(counts[i]) == expected[ids[i]][int(steps[i])], (i, ids[i], steps[i])
    # every simulation's requests took its steps in arrival order
    for j in range(6):
        mine = steps[ids == j]
        assert sorted(mine.tolist()) == list(range(1, per_sim + 1))
        assert np.all(np.diff(steps[np.argsort(arr)][ids[np.argsort(arr)] == j].astype(int)) > 0)
    # final device state equals the reference after per_sim steps (the
    # incremental policy writes it back on request)
    for j in range(6):
        sv.export(j)
    for (inst, side, sigma, seed), g in zip(sims, states):
        *_, (st, ul, uh, sl, sh) = list(walk.walk(inst.upd_lo, inst.sub_lo, side, sigma, seed,
                                                  per_sim))
        assert np.array_equal(g[0].cpu().numpy(), ul) and np.array_equal(g[3].cpu().numpy(), sh)
    sv.close()
    # alone: each simulation served on its own from the initial state
    for j, s in enumerate(sims):
        sv1, _ = _server(ddm, [s], policy)
        c1, st1, _, _ = sv1.run(np.zeros(per_sim, np.int32), np.arange(per_sim) * 1e-4)
        assert [int(c) for c in c1] == [expected[j][k] for k in range(1, per_sim + 1)]
        assert st1.tolist() == list(range(1, per_sim + 1))
        sv1.close()


def test_tight_budget_admission(ddm, oracle):
    """An arena that holds little more than the largest single request: groups
    are cut to fit, results stay exact, and the peak stays within budget."""
    sims = _small_sims(5, seed=4)
    expected = [_expected_counts(oracle, *s, 3) for s in sims]
    probe, _ = _server(ddm, sims[:1])
    probe.close()
    from paper_1703_06680_amd.ddm import library
    need = max(library().ddm_workspace_bytes(s[0].n, s[0].m, 2, 0, 0) for s in sims)
    arena = int(need * 1.6) + (1 << 20)
    sv, _ = _server(ddm, sims, arena=arena, slots=3, max_batch=5)
    ids = np.tile(np.arange(5, dtype=np.int32), 3)
    arr = np.zeros(ids.size)  # all at once: admission decides
    counts, steps, lat, stats = sv.run(ids, arr)
    for i in range(ids.size):
        assert int(counts[i]) == expected[ids[i]][int(steps[i])]
    assert stats["peak_arena_bytes"] <= arena
    sv.close()


def test_server_rejects_bad_requests(ddm):
    sims = _small_sims(2, seed=5)
    sv, _ = _server(ddm, sims)
    with pytest.raises(ddm.DDMError) as e:
        sv.run(np.array([0, 5], np.int32), np.array([0.0, 0.0]))
    assert e.value.code == ddm.DDM_E_INVAL
    with pytest.raises(ddm.DDMError) as e:
        sv.run(np.array([0], np.int32), np.array([-1.0]))
    assert e.value.code == ddm.DDM_E_INVAL
    sv.close()
    inst = sims[0][0]
    need = ddm.library().ddm_workspace_bytes(inst.n, inst.m, 2, 0, 0)
    small = ddm.Server((need // 2) & ~255, policy="batched")
    with pytest.raises(ddm.DDMError) as e:
        small.add_sim(*_upload(inst), 1.0, 0.1, 1)
    assert e.value.code == ddm.DDM_E_WORKSPACE
    small.close()


def test_served_d3_and_invalid_state(ddm, oracle):
    """d = 3 simulations are served exactly; a simulation whose state holds a
    NaN makes its request fail with DDM_E_INVAL while the others still
    count."""
    sims = W.serving_sims(3, d=3, seed=12, lo=2_000, hi=9_000)
    expected = [_expected_counts(oracle, *s, 2) for s in sims]
    sv, states = _server(ddm, sims, max_batch=3)
    ids = np.array([0, 1, 2, 0, 1, 2], np.int32)
    counts, steps, _, _ = sv.run(ids, np.zeros(6))
    for i in range(6):
        assert int(counts[i]) == expected[ids[i]][int(steps[i])]
    states[1][0][7, 2] = float("nan")  # poison simulation 1
    with pytest.raises(ddm.DDMError) as e:
        sv.run(np.array([1], np.int32), np.zeros(1))
    assert e.value.code == ddm.DDM_E_INVAL
    sv.close()
