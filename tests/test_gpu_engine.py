"""Serving engine (ppn_engine_*): resident scenes stepped on request.

* Each result is bit-identical alone and in the mix: the same requests run one
  scene at a time on one worker, all at once on several workers (their kernels
  overlapping on the device), with their PCG solves batched into shared
  launches (one precision at a time, and FP64 and mixed-form scenes together),
  and through the single-scene API.
* Admission by footprint: with a budget for two scenes, four scenes take turns
  in device memory (evictions keep the state on the host) with unchanged results.
* Against the FP64 oracle: rotated blocks of the batched workload, stepped in the
  mixed form through the engine, per scene (positions and residual as in the
  mixed-precision tests).
"""
import numpy as np
import pytest

import oracle
from paper_2505_21013_amd import PPN_FP64, PPN_MIXED, Engine, run_steps
from scenes import batch_scenes

from helpers import gpu_scene

pytestmark = pytest.mark.gpu


def _small_scenes(k, max_tets=12000):
    out = [s for s in batch_scenes() if s.n_tets <= max_tets]
    return out[:k]


def _run(engine, scenes, ids, n_steps, mode="PPN", interleave=True):
    """Submit n_steps requests per scene (all at once if interleave, else one
    scene after the other, waiting for each request); return per-scene stats."""
    stats = {i: [] for i in range(len(scenes))}
    if interleave:
        reqs = []
        for n in range(1, n_steps + 1):
            for i, (sc, sid) in enumerate(zip(scenes, ids)):
                reqs.append((i, engine.ppn_engine_submit(sid, mode, sc.targets(n))))
        for i, r in reqs:
            stats[i].append(engine.ppn_engine_wait(r))
    else:
        for i, (sc, sid) in enumerate(zip(scenes, ids)):
            for n in range(1, n_steps + 1):
                stats[i].append(engine.ppn_engine_wait(engine.ppn_engine_submit(sid, mode, sc.targets(n))))
    states = [engine.ppn_engine_get_state(sid, sc.n_verts) for sc, sid in zip(scenes, ids)]
    return stats, states


KEYS = ("status", "newton_iters", "pcg_iters", "projected", "inner_rounds", "res_l2")


def test_engine_results_identical_alone_and_in_mix():
    scenes = _small_scenes(6)
    with Engine(n_workers=1) as e1:
        ids1 = [e1.add_scene(sc) for sc in scenes]
        alone, st_alone = _run(e1, scenes, ids1, 3, interleave=False)
    with Engine(n_workers=6) as e6:
        ids6 = [e6.add_scene(sc) for sc in scenes]
        mix, st_mix = _run(e6, scenes, ids6, 3, interleave=True)
        info = e6.ppn_engine_get_info()
    assert info["resident_scenes"] == len(scenes) and info["evictions"] == 0
    for i in range(len(scenes)):
        assert all(s["status"] == "PPN_OK" for s in alone[i]), scenes[i].name
        for a, b in zip(alone[i], mix[i]):
            assert all(a[k] == b[k] for k in KEYS), (scenes[i].name, a, b)
        assert np.array_equal(st_alone[i][0], st_mix[i][0]) and np.array_equal(st_alone[i][1], st_mix[i][1])
    # and the same as the single-scene API
    for i, sc in enumerate(scenes[:2]):
        g = gpu_scene(sc)
        run_steps(g, sc, "PPN", 3)
        x, v = g.ppn_get_state()
        g.close()
        assert np.array_equal(x, st_mix[i][0]) and np.array_equal(v, st_mix[i][1])


@pytest.mark.parametrize("precision", [PPN_FP64, PPN_MIXED])
def test_engine_pcg_batching_changes_nothing(precision):
    """Solves of scenes stepped at the same time share launches; every scene's
    bits stay those of its unbatched run."""
    scenes = _small_scenes(6)
    with Engine(n_workers=1) as e1:
        ids1 = [e1.add_scene(sc, precision=precision) for sc in scenes]
        alone, st_alone = _run(e1, scenes, ids1, 3, interleave=False)
    with Engine(n_workers=6) as eb:
        eb.ppn_engine_set_pcg_batching(True)
        idsb = [eb.add_scene(sc, precision=precision) for sc in scenes]
        mix, st_mix = _run(eb, scenes, idsb, 3, interleave=True)
        info = eb.ppn_engine_get_info()
    n_solves = sum(s["solves"] for st in mix.values() for s in st)
    assert info["pcg_batches"] > 0 and info["pcg_batched_solves"] >= n_solves > 0, info
    for i in range(len(scenes)):
        for n, (a, b) in enumerate(zip(alone[i], mix[i])):
            diff = {k: (a[k], b[k]) for k in KEYS if a[k] != b[k]}
            assert not diff, (scenes[i].name, n + 1, diff)
        assert np.array_equal(st_alone[i][0], st_mix[i][0]) and np.array_equal(st_alone[i][1], st_mix[i][1])


@pytest.mark.parametrize("precision", [PPN_FP64, PPN_MIXED])
def test_engine_evaluation_batching_changes_nothing(precision):
    """With PPN_BATCH_EVAL the scenes' evaluation phases (element quantities,
    assembly, gradient norms) and line-search launches are shared too: every
    scene keeps the bits of its run alone, and of its run alone without graphs."""
    scenes = _small_scenes(6)
    with Engine(n_workers=1) as e1:
        ids1 = [e1.add_scene(sc, precision=precision, params=dict(use_graphs=0)) for sc in scenes]
        alone, st_alone = _run(e1, scenes, ids1, 3, interleave=False)
    with Engine(n_workers=6) as eb:
        eb.ppn_engine_set_batching(pcg=True, evaluation=True)
        idsb = [eb.add_scene(sc, precision=precision) for sc in scenes]
        mix, st_mix = _run(eb, scenes, idsb, 3, interleave=True)
        info = eb.ppn_engine_get_info()
    n_iters = sum(s["newton_iters"] for st in mix.values() for s in st)
    assert info["eval_launches"] > 0 and info["eval_batched_phases"] >= n_iters, info
    for i in range(len(scenes)):
        for n, (a, b) in enumerate(zip(alone[i], mix[i])):
            diff = {k: (a[k], b[k]) for k in KEYS if a[k] != b[k]}
            assert not diff, (scenes[i].name, n + 1, diff)
        assert np.array_equal(st_alone[i][0], st_mix[i][0]) and np.array_equal(st_alone[i][1], st_mix[i][1])


def test_engine_pcg_batching_mixed_precisions_together():
    """FP64 and mixed-form scenes in one batching engine: the batcher runs its
    FP64-matrix and FP32-matrix lanes side by side, and every scene keeps the
    bits of its unbatched run in its own precision."""
    scenes = _small_scenes(6)
    precs = [PPN_FP64 if i % 2 == 0 else PPN_MIXED for i in range(len(scenes))]
    with Engine(n_workers=1) as e1:
        ids1 = [e1.add_scene(sc, precision=p) for sc, p in zip(scenes, precs)]
        alone, st_alone = _run(e1, scenes, ids1, 3, interleave=False)
    with Engine(n_workers=6) as eb:
        eb.ppn_engine_set_pcg_batching(True)
        idsb = [eb.add_scene(sc, precision=p) for sc, p in zip(scenes, precs)]
        mix, st_mix = _run(eb, scenes, idsb, 3, interleave=True)
        info = eb.ppn_engine_get_info()
    assert info["pcg_batches"] > 0, info
    for i in range(len(scenes)):
        for n, (a, b) in enumerate(zip(alone[i], mix[i])):
            diff = {k: (a[k], b[k]) for k in KEYS if a[k] != b[k]}
            assert not diff, (scenes[i].name, precs[i], n + 1, diff)
        assert np.array_equal(st_alone[i][0], st_mix[i][0]) and np.array_equal(st_alone[i][1], st_mix[i][1])


def test_engine_footprint_is_device_bytes():
    sc = _small_scenes(1)[0]
    with Engine(n_workers=1) as e:
        for prec in (PPN_FP64, PPN_MIXED):
            sid = e.add_scene(sc, precision=prec)
            g = gpu_scene(sc, precision=prec)
            assert e.ppn_engine_scene_footprint(sid) == g.ppn_scene_info()["device_bytes"]
            g.close()


def test_engine_admission_by_footprint():
    scenes = _small_scenes(4)
    with Engine(n_workers=4) as ref:
        rid = [ref.add_scene(sc) for sc in scenes]
        want, st_want = _run(ref, scenes, rid, 3)
    with Engine(n_workers=1) as probe:
        fp = [probe.ppn_engine_scene_footprint(probe.add_scene(sc)) for sc in scenes]
    budget = sum(sorted(fp)[-2:])  # room for the two largest at a time
    with Engine(n_workers=4, mem_budget_bytes=budget) as e:
        ids = [e.add_scene(sc) for sc in scenes]
        got, st_got = _run(e, scenes, ids, 3)
        info = e.ppn_engine_get_info()
    assert info["evictions"] > 0 and info["resident_bytes"] <= budget
    for i in range(len(scenes)):
        for a, b in zip(want[i], got[i]):
            assert all(a[k] == b[k] for k in KEYS), scenes[i].name
        assert np.array_equal(st_want[i][0], st_got[i][0])


def test_engine_request_record_is_freed_after_its_wait():
    """A request is waited on once: its record is freed then, so a second wait on
    the same id is an argument error, while other requests are unaffected."""
    from paper_2505_21013_amd import PPNError
    sc = _small_scenes(1)[0]
    with Engine(n_workers=1) as e:
        sid = e.add_scene(sc)
        r1 = e.ppn_engine_submit(sid, "PPN", sc.targets(1))
        r2 = e.ppn_engine_submit(sid, "PPN", sc.targets(2))
        assert e.ppn_engine_wait(r1)["status"] == "PPN_OK"
        with pytest.raises(PPNError) as ei:
            e.ppn_engine_wait(r1)
        assert ei.value.code == -1
        assert e.ppn_engine_wait(r2)["status"] == "PPN_OK"
        with pytest.raises(PPNError):
            e.ppn_engine_wait(r2 + 1000)


def test_engine_oversized_scene_is_refused():
    sc = _small_scenes(1)[0]
    with Engine(n_workers=1, mem_budget_bytes=1 << 16) as e:
        sid = e.add_scene(sc)
        assert e.ppn_engine_scene_footprint(sid) > 1 << 16
        r = e.ppn_engine_wait(e.ppn_engine_submit(sid, "PPN", sc.targets(1)))
    assert r["status"] == "PPN_ERR_OOM"


def test_engine_batch_against_oracle_mixed():
    scenes = _small_scenes(4, max_tets=3000)
    n_steps = 3
    with Engine(n_workers=4) as e:
        ids = [e.add_scene(sc, precision=PPN_MIXED) for sc in scenes]
        reqs = [[e.ppn_engine_submit(sid, "PPN", sc.targets(n)) for n in range(1, n_steps + 1)]
                for sc, sid in zip(scenes, ids)]
        stats = [[e.ppn_engine_wait(r) for r in rs] for rs in reqs]
        states = [e.ppn_engine_get_state(sid, sc.n_verts) for sc, sid in zip(scenes, ids)]
    for sc, st, (x, v) in zip(scenes, stats, states):
        orc_x = []
        _, ost = oracle.run_scene(sc, "PPN", n_steps=n_steps,
                                  callback=lambda n, s, o: orc_x.append(s.x.copy()))
        diag = float(np.linalg.norm(sc.X.max(0) - sc.X.min(0)))
        assert all(s["status"] == "PPN_OK" for s in st) and all(o.converged for o in ost), sc.name
        assert float(np.max(np.abs(x - orc_x[-1]))) <= 1e-6 * diag, sc.name
        for g, o in zip(st, ost):
            assert abs(g["res_l2"] - o.res_l2) <= 1e-6 * o.res0_l2, sc.name
