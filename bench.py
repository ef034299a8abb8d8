#!/usr/bin/env python3
"""Benchmark: PPN backward-Euler time steps per second on one MI355X.

Workload (default): cube of 64^3 hex cells split into 1,572,864 linear tets
(274,625 vertices), Stable Neo-Hookean with E log-uniform in [1e4, 1e6] Pa per
element, nu = 0.48, rho = 1000, dt = 1/30 s, gravity, bottom face pinned and top
face pushed down 60% over 50 steps; PPN (Algorithm 1) in FP64; stop when the
Newton velocity step is below 1e-3 m/s.  Inputs are seeded and synthetic.
The timed window is steps 1..20 of that schedule (24% compression), where PN,
PDN and PPN all converge; from about step 28 on no mode converges within 100
Newton iterations at this resolution (the scene buckles).

A "step" is one time step (a full Newton minimisation through every stage of
the hot path).  W warm-up steps run first on the same scene, the state is then
reset to the initial one, and K steps (1..K of the schedule) are timed between
two device synchronisations.  All data are resident in HBM before timing.

Printed as one JSON line: steps/s (value), per-step latency p50/p99, in-situ
eigen-projections/s, the roofline of the dominant kernel (the PCG matrix
product, timed live with HIP events on the scene stream) and the oracle's CPU
baseline on a bounded sample of the same workload.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def spmv_bytes(N, NB, fp32=False):
    """Algorithmic bytes of one PCG matrix-product launch.  The symmetric matrix
    is stored once (half storage): every stored block, the N diagonal and the
    E = (NB - N) / 2 edge blocks, is read once (72 B; 36 B for the FP32 matrix
    of the mixed form); every block of the full pattern costs its column and
    value reference (8 B); each 64-row group its slot count (4 B).  Per vertex,
    FP64: its 48-byte (z, d_old) record gathered once, the new direction and
    the product written (24 B each); mixed form: its 24-byte FP32 record
    gathered once, its own FP64 z and d_old read (24 B each), the new direction
    and the product written."""
    E = (NB - N) // 2
    per_vertex = 5 * 24 if fp32 else 4 * 24
    return 8 * NB + (36 if fp32 else 72) * (N + E) + 4 * ((N + 63) // 64) + per_vertex * N


def measured_traffic(fp32=False):
    """HBM bytes per matrix-product launch from the committed counter summary,
    valid only while the kernel source is the one the counters were taken on."""
    import hashlib
    import re
    prof = os.path.join(ROOT, "profiles", "k_pcg_spmv_cube64_compress_ppn_%s.md" % ("mixed" if fp32 else "fp64"))
    src = os.path.join(ROOT, "paper_2505_21013_amd", "csrc", "k_pcg.hip")
    try:
        text = open(prof).read()
        want = re.search(r"sha256\[:16\] = ([0-9a-f]{16})", text).group(1)
        value = float(re.search(r"traffic_bytes_per_launch: (\d+)", text).group(1))
        have = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except (OSError, AttributeError):
        return None
    return value if have == want else None


# The extrapolation checked against whole oracle time steps of the 1.57M-tet
# cube (tests/golden/cube64_compress_PPN.json records each step's oracle time;
# both were taken on the same host, an Intel Xeon at 2.7 GHz): the sampled
# costs with those steps' counts give 730.2 and 423.0 s against 563.6 and
# 326.5 s timed, i.e. the extrapolation overestimates a step by 1.30x.
EXTRAPOLATION_CHECK = {"extrapolated_over_timed": 1.30, "steps": "1 and 2 of the 1.57M-tet cube",
                       "host": "Intel(R) Xeon(R) Processor @ 2.70GHz, one core"}


def cpu_baseline(cfg, per_step_counts):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    core = min(os.sched_getaffinity(0))
    r = subprocess.run([sys.executable, "-m", "oracle.baseline", "--config", str(cfg), "--cpu", str(core)],
                       cwd=ROOT, capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    c = json.loads(r.stdout.strip().splitlines()[-1])
    from oracle.baseline import per_step_seconds
    sec = per_step_seconds(c, per_step_counts)
    return {"value": 1.0 / sec, "unit": "steps/s", "cores": c["threads"], "kind": "oracle",
            "sample": (f"FP64 NumPy oracle, 1 thread, on the same workload: element evaluation + "
                       f"assembly of {c['n_sample']} elements, clamping of {c['n_proj']} element "
                       f"Hessians, {c['pcg_iters_timed']} PCG iterations on the partial operator and one "
                       f"line-search energy pass, timed ({c['wall_s']:.1f} s) and scaled per element / per "
                       f"nonzero to the full mesh with the timed run's mean per-step counts"),
            "s_per_step": sec, "cpu_model": c.get("cpu_model"), "pinned_core": c.get("pinned_core"),
            "host_cpus": c.get("host_cpus"), "extrapolation_check": EXTRAPOLATION_CHECK}


def form_params(a):
    """Scene parameters the command line overrides (None: the defaults)."""
    prm = {}
    if a.no_graphs:
        prm["use_graphs"] = 0
    if a.pcg_load_mode is not None:
        prm["pcg_load_mode"] = a.pcg_load_mode
    if a.eps_clamp is not None:
        prm["eps_clamp"] = a.eps_clamp
    return prm or None


def run_form(a, precision, torch, np):
    """Warm-up steps, reset to the initial state, then K timed steps."""
    from paper_2505_21013_amd import PPN_FP64, PPN_MIXED, scene_from
    from scenes import config, cube_compress
    sc = cube_compress(n=a.cells) if a.cells and a.config == 2 else config(a.config)
    stream = torch.cuda.current_stream().cuda_stream
    s = scene_from(sc, stream=stream, precision=PPN_MIXED if precision == "mixed" else PPN_FP64,
                   params=form_params(a))
    info = s.ppn_scene_info()
    for n in range(1, a.warmup + 1):
        s.ppn_set_dirichlet(sc.dirichlet_ids, sc.targets(n))
        st = s.ppn_newton_step(a.mode)
        print(f"[{precision}] warmup {n}: {st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    s.ppn_set_state(sc.x0, sc.v0)
    s.ppn_set_profiling(True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(1, a.steps + 1):
        ts = time.perf_counter()
        s.ppn_set_dirichlet(sc.dirichlet_ids, sc.targets(n))
        st = s.ppn_newton_step(a.mode)
        st["wall_ms"] = (time.perf_counter() - ts) * 1e3
        stats.append(st)
        print(f"[{precision}] step {n}: {st['wall_ms']:.1f} ms newton {st['newton_iters']} "
              f"pcg {st['pcg_iters']} projected {st['projected']} {st['status']}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    x = s.ppn_get_positions()
    # Eigen-projection rate on full passes over all elements (the PN path):
    # one extra PN step after the timed region, outside the timing.
    xs, vs = s.ppn_get_state()
    s.ppn_set_dirichlet(sc.dirichlet_ids, sc.targets(a.steps + 1))
    pn = s.ppn_newton_step("PN")
    s.ppn_set_state(xs, vs)
    s.close()
    full_pass = {"projections_per_s": pn["projected"] / (pn["ms_eig"] * 1e-3) if pn["ms_eig"] > 0 else None,
                 "projected": pn["projected"], "ms_eig": pn["ms_eig"],
                 "passes": pn["projected"] / max(info["n_tets"], 1)}
    tot = {k: sum(st[k] for st in stats) for k in
           ("newton_iters", "pcg_iters", "solves", "projected", "ms_eig", "ms_spmv", "n_spmv",
            "ls_backtracks", "inner_rounds", "refine_rounds", "ms_pcg")}
    return {"elapsed": elapsed, "stats": stats, "tot": tot, "info": info, "x": x, "X": sc.X,
            "eig_full_pass": full_pass}


def summary(R, K, info, np):
    lat = np.array([st["wall_ms"] for st in R["stats"]])
    tot = R["tot"]
    return {
        "p50_step_ms": float(np.percentile(lat, 50)),
        "p99_step_ms": float(np.percentile(lat, 99)),
        "eig_projections_per_s": (tot["projected"] / (tot["ms_eig"] * 1e-3)) if tot["ms_eig"] > 0 else None,
        "eig_projections_per_s_full_pass": R["eig_full_pass"]["projections_per_s"],
        "per_step": {"newton_iters": tot["newton_iters"] / K, "pcg_iters": tot["pcg_iters"] / K,
                     "solves": tot["solves"] / K, "projected": tot["projected"] / K,
                     "proj_ratio": tot["projected"] / max(tot["newton_iters"] * info["n_tets"], 1),
                     "ls_backtracks": tot["ls_backtracks"] / K},
        "all_steps_converged": all(st["status"] == "PPN_OK" for st in R["stats"]),
    }


def composite_roofline(R, precision, info, K):
    """Time a step would take if every part of the hot path ran at its roofline
    (HBM bytes / 8 TB/s, eigensolves at the FP64 / FP32 vector peak), with the
    part counts of the timed run, against the measured step time.  Algorithmic
    bytes per unit, as the kernels move them:
      element evaluation + assembly, per Newton iteration: 1592 B per tet
        (152 B of element data read, 720 B of slots written, slots read back
        once by the vertex and edge passes), 261 B per vertex, 76 B per edge
        (its block written once, its slot range pointer);
      PCG iteration: the matrix product (spmv_bytes) + the update (240 B per
        vertex: q, d, r, x and the 6-entry symmetric block-Jacobi inverse read,
        x, r and the 48-byte (z, d) record that the next product gathers
        written; 216 B with the FP32 inverse);
      line-search pass (four step sizes): 112 B per tet + 84 B per vertex;
      eigen-projection: 45.6 kflop (measured executed flops of the 9x9 Jacobi)."""
    N, T, NB = info["n_verts"], info["n_tets"], info["n_blocks"]
    E = (NB - N) // 2
    tot = R["tot"]
    fp32 = precision == "mixed"
    bw = HBM_PEAK_GBS * 1e9
    pcg = tot["pcg_iters"] * (spmv_bytes(N, NB, fp32) + (216 if fp32 else 240) * N) / bw
    elem = tot["newton_iters"] * (1592 * T + 261 * N + 76 * E) / bw
    ls = (tot["newton_iters"] + tot["ls_backtracks"] / 4.0) * (112 * T + 84 * N) / bw
    eig = tot["projected"] * 45.6e3 / ((157.3 if fp32 else 78.6) * 1e12)
    t_roof = (pcg + elem + ls + eig) / K
    t_meas = R["elapsed"] / K
    ms = lambda t: t / K * 1e3
    return {"t_roof_ms": t_roof * 1e3, "t_measured_ms": t_meas * 1e3, "frac": t_roof / t_meas,
            "parts_roof_ms": {"pcg": ms(pcg), "element_assembly": ms(elem), "line_search": ms(ls),
                              "eigensolve": ms(eig)},
            "parts_measured_ms": {"pcg": tot["ms_pcg"] / K, "eigensolve": tot["ms_eig"] / K}}


def roofline(R, precision, info, cfg):
    tot = R["tot"]
    fp32 = precision == "mixed"
    spmv_avg_s = tot["ms_spmv"] / max(tot["n_spmv"], 1) * 1e-3
    bytes_launch = spmv_bytes(info["n_verts"], info["n_blocks"], fp32)
    achieved = bytes_launch / spmv_avg_s / 1e9 if spmv_avg_s > 0 else 0.0
    traffic = measured_traffic(fp32) if cfg == 2 else None
    return {"kernel": "k_pcg_spmv (PCG matrix product, %s BCSR 3x3)" % ("FP32" if fp32 else "FP64"),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "bytes_per_launch": bytes_launch, "avg_launch_us": spmv_avg_s * 1e6,
            "launches": tot["n_spmv"]}


def _engine_scenes(engine, scenes, precision, graphs=True):
    from paper_2505_21013_amd import PPN_MIXED
    t = time.perf_counter()
    prm = None if graphs else dict(use_graphs=0)
    ids = [engine.add_scene(sc, precision=PPN_MIXED if precision == "mixed" else 0, params=prm) for sc in scenes]
    print(f"registered {len(ids)} scenes in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    return ids


def run_batch(a):
    """64 independent scenes (rotated cubes and beams of 24..257k tets), mixed
    form, K steps each, through the engine: one worker (scenes one after the
    other), --workers workers (scenes overlapping on the device), and one
    worker per scene with the PCG solves batched into shared launches."""
    import numpy as np
    import torch
    from paper_2505_21013_amd import Engine
    from scenes import batch_scenes
    torch.cuda.set_device(0)
    scenes = batch_scenes()
    K = min(a.steps, 20)
    out = {"metric": "batched time steps/s (64 independent scenes, mixed form)", "unit": "steps/s",
           "n_gpus": 1, "steps_per_scene": K, "dtype": "f32+f64", "data": "synthetic",
           "higher_is_better": True,
           "config": {"workload": f"64 rotated blocks, {sum(s.n_tets for s in scenes)} tets in total "
                                  f"({min(s.n_tets for s in scenes)}..{max(s.n_tets for s in scenes)} per "
                                  f"scene), steps 1..{K}, PPN", "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")}}
    # (key, workers, batching: 0 none / 1 PCG / 2 PCG + evaluation and line search, graphs)
    runs = [("workers_1", 1, 0, True), (f"workers_{a.workers}_no_graphs", a.workers, 0, False),
            (f"workers_{a.workers}", a.workers, 0, True), ("batched_pcg", len(scenes), 1, True),
            ("batched_pcg_eval", len(scenes), 2, True)]
    for key, workers, batched, graphs in runs:
        with Engine(n_workers=workers) as e:
            if batched:
                e.ppn_engine_set_batching(pcg=True, evaluation=batched == 2)
            ids = _engine_scenes(e, scenes, "mixed", graphs)
            warm = [e.ppn_engine_submit(sid, "PPN", sc.targets(1)) for sc, sid in zip(scenes, ids)]
            for r in warm:
                e.ppn_engine_wait(r)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reqs = [e.ppn_engine_submit(sid, "PPN", sc.targets(n)) for n in range(2, K + 2)
                    for sc, sid in zip(scenes, ids)]
            res = [e.ppn_engine_wait(r) for r in reqs]
            el = time.perf_counter() - t0
            info = e.ppn_engine_get_info()
            ok = all(r["status"] in ("PPN_OK",) for r in res)
            out[key] = {"workers": workers, "pcg_batching": batched >= 1, "eval_batching": batched == 2,
                        "graphs": graphs and batched < 2, "value": len(reqs) / el,
                        "elapsed_s": el, "all_converged": ok,
                        "newton_iters": sum(r["newton_iters"] for r in res),
                        "pcg_iters": sum(r["pcg_iters"] for r in res),
                        "mean_step_ms": sum(r["ms_total"] for r in res) / len(res),
                        "mean_step_pcg_ms": sum(r["ms_pcg"] for r in res) / len(res)}
            if batched:
                out[key]["pcg_chunks"] = info["pcg_batches"]
                out[key]["pcg_solves"] = info["pcg_batched_solves"]
            if batched == 2:
                out[key]["eval_launches"] = info["eval_launches"]
                out[key]["eval_phases"] = info["eval_batched_phases"]
            print(f"batch {key}: {len(reqs) / el:.1f} steps/s", file=sys.stderr, flush=True)
    out["value"] = max(out[k]["value"] for k, _, _, _ in runs)
    out["speedup_vs_one_worker"] = out["value"] / out["workers_1"]["value"]
    return out


def run_serve(a):
    """Serving loop: 128 resident scenes (1e3..5e5 tets, ~10M in total), one
    warm-up step each, then --requests time-step requests with exponential
    inter-arrival gaps (mean 1/--rate) on uniformly drawn scenes, submitted in
    real time; latency = completion - arrival.  PCG solves of concurrently
    stepped scenes are batched unless --no-pcg-batching."""
    import numpy as np
    import torch
    from paper_2505_21013_amd import Engine
    from scenes import serving_scenes
    torch.cuda.set_device(0)
    scenes = serving_scenes()
    rng = np.random.default_rng(4)
    gaps = rng.exponential(1.0 / a.rate, size=a.requests)
    which = rng.integers(len(scenes), size=a.requests)
    batching = not a.no_pcg_batching
    with Engine(n_workers=a.workers) as e:
        if batching:
            e.ppn_engine_set_pcg_batching(True)
        ids = _engine_scenes(e, scenes, "mixed")
        step = [1] * len(scenes)
        warm = [e.ppn_engine_submit(sid, "PPN", sc.targets(1)) for sc, sid in zip(scenes, ids)]
        for r in warm:
            e.ppn_engine_wait(r)
        info0 = e.ppn_engine_get_info()
        print(f"warm: {info0}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        due = t0
        reqs, tags = [], []
        for g, k in zip(gaps, which):
            due += g
            now = time.perf_counter()
            if due > now:
                time.sleep(due - now)
            step[k] += 1
            reqs.append(e.ppn_engine_submit(ids[k], "PPN", scenes[k].targets(step[k])))
            tags.append((scenes[k].name, int(scenes[k].n_tets), step[k]))
        res = [e.ppn_engine_wait(r) for r in reqs]
        el = time.perf_counter() - t0
        info = e.ppn_engine_get_info()
    lat = np.array([r["latency_ms"] for r in res])
    que = np.array([r["queue_ms"] for r in res])
    return {"metric": "served time-step requests/s; p50/p99 request latency (1 GPU)",
            "value": len(res) / el, "unit": "requests/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": f"{len(scenes)} resident cubes, {sum(s.n_tets for s in scenes)} tets "
                                   f"({min(s.n_tets for s in scenes)}..{max(s.n_tets for s in scenes)}), "
                                   f"{a.requests} requests, Poisson {a.rate:g}/s, one PPN step each",
                       "workers": a.workers, "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
                       "pcg_batching": batching},
            "offered_rate": a.rate, "elapsed_s": el,
            "p50_latency_ms": float(np.percentile(lat, 50)), "p99_latency_ms": float(np.percentile(lat, 99)),
            "p50_queue_ms": float(np.percentile(que, 50)), "p99_queue_ms": float(np.percentile(que, 99)),
            "all_ok": all(r["status"] in ("PPN_OK", "PPN_WARN_NOT_CONVERGED") for r in res),
            "not_converged": sum(r["status"] != "PPN_OK" for r in res),
            "not_converged_requests": [{"scene": t[0], "tets": t[1], "step": t[2], "status": r["status"],
                                        "newton_iters": r["newton_iters"]}
                                       for t, r in zip(tags, res) if r["status"] != "PPN_OK"],
            "resident_bytes": info["resident_bytes"], "resident_scenes": info["resident_scenes"],
            "evictions": info["evictions"]}


def run_eig(a):
    """Eigen-projection microbenchmark on harvested matrices: the element
    Hessians of the twisted beam at step 90 of its 100-step schedule (all
    122,880 elements) and of the compressed cube at step 20 (262,144 elements
    at a fixed stride), evaluated by the library at the PPN state it reached,
    then projected in device memory by the stateless batch projector (FP64,
    eps 1e-8).  Median of 5 launches, timed with events on its stream."""
    import numpy as np
    import torch
    from paper_2505_21013_amd import ppn_project_batch_dev, run_steps, scene_from
    from scenes import config
    torch.cuda.set_device(0)
    st = torch.cuda.current_stream()
    rows = []
    for name, k, n_steps, sample in (("beam 80x16x16 twist, step 90", 1, 90, None),
                                     ("cube 64^3 compression, step 20", 2, 20, 262144)):
        sc = config(k)
        s = scene_from(sc, stream=st.cuda_stream)
        run_steps(s, sc, "PPN", n_steps)
        x, _ = s.ppn_get_state()
        ids = None if sample is None else np.linspace(0, sc.n_tets - 1, sample).astype(np.int32)
        H = s.ppn_eval_element_hessians(x, ids)
        s.close()
        n = H.shape[0]
        lam = np.linalg.eigvalsh(H[:: max(1, n // 20000)])
        Hd = torch.from_numpy(np.ascontiguousarray(H.reshape(n, 144))).cuda()
        out = torch.empty_like(Hd)
        ppn_project_batch_dev(Hd, out, n, 1e-8, st.cuda_stream)
        times = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            ppn_project_batch_dev(Hd, out, n, 1e-8, st.cuda_stream)
            e1.record(st)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        t = float(np.median(times))
        # indefinite: an eigenvalue below -1e-8 of the spectral radius (the three translation
        # modes are zero up to rounding)
        indef = lam[:, 0] < -1e-8 * np.abs(lam).max(axis=1)
        rows.append({"source": name, "matrices": n, "share_indefinite": float(indef.mean()),
                     "ms_per_batch": t * 1e3, "projections_per_s": n / t})
        print(f"[eig] {name}: {n} matrices, {n / t:.3e} projections/s", file=sys.stderr, flush=True)
    return {"metric": "12x12 eigen-projections/s on harvested element Hessians (FP64, batch projector, 1 GPU)",
            "value": min(r["projections_per_s"] for r in rows), "unit": "projections/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic", "rows": rows}


def run_ablation(a):
    """Variants of the paper on the compressed heterogeneous cube at 32^3 cells
    (196,608 tets, FP64): steps 1..20 of the 50-step schedule in PPN give a
    state at 24% compression with indefinite elements; from that state each
    variant runs steps 21..30.  (The twisted beam is no use here: its global
    Hessian stays positive definite through the schedule, so PPN and PDN never
    project.)  Reported per variant: Newton and PCG iterations, projected
    element Hessians and wall time."""
    import numpy as np
    import torch
    from paper_2505_21013_amd import run_steps, scene_from
    from scenes import cube_compress
    torch.cuda.set_device(0)
    sc = cube_compress(n=32)
    stream = torch.cuda.current_stream().cuda_stream
    s = scene_from(sc, stream=stream)
    run_steps(s, sc, "PPN", 20)
    x0, v0 = s.ppn_get_state()
    variants = [("PPN", dict(alpha=al, beta=be)) for al in (0.25, 0.5, 0.75) for be in (1.0, 2.0, 4.0)]
    variants += [("PDN", dict(pdn_countdown=c)) for c in (1, 4, 8)]
    variants += [("PN", {})]
    variants += [(m, dict(eig_mirror=1)) for m in ("PN", "PDN", "PPN")]
    rows = []
    for mode, kw in variants:
        s.ppn_set_params(stop_mode=sc.stop_mode, stop_tol=sc.stop_tol, **kw)
        s.ppn_set_state(x0, v0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = run_steps(s, sc, mode, 10, first_step=21)
        el = time.perf_counter() - t0
        rows.append({"mode": mode, **kw, "newton_iters": sum(q["newton_iters"] for q in st),
                     "pcg_iters": sum(q["pcg_iters"] for q in st), "projected": sum(q["projected"] for q in st),
                     "converged_steps": sum(q["status"] == "PPN_OK" for q in st), "seconds": el})
        print(rows[-1], file=sys.stderr, flush=True)
    s.close()
    return {"metric": "paper variants on the compressed cube, steps 21..30 from one state (FP64)",
            "config": {"workload": f"cube 32^3 cells -> {sc.n_tets} tets, E log-uniform [1e4,1e6], nu 0.48, "
                                   "top pushed down 60% over 50 steps, state after 20 PPN steps"},
            "rows": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, help="workload index (2 = 1.57M-tet cube)")
    ap.add_argument("--mode", default="PPN", choices=["PN", "PDN", "PPN"])
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"],
                    help="fp64 or mixed alone, or both (FP64 headline, mixed reported beside it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graphs", action="store_true",
                    help="plain launches instead of the captured evaluation graph (use_graphs = 0)")
    ap.add_argument("--pcg-load-mode", type=int, default=None, choices=[0, 1, 2],
                    help="force how the PCG product loads the matrix (0 small, 1 cache-resident, "
                         "2 streamed; default: chosen from its size)")
    ap.add_argument("--eps-clamp", type=float, default=None,
                    help="eigenvalue clamp eps (default 1e-8, Sec. 5.1); the level the projection lifts the "
                         "negative and the three translational zero eigenvalues to")
    ap.add_argument("--cells", type=int, default=None,
                    help="compressed cube of N^3 cells instead of 64^3 (size studies: no CPU baseline, and no "
                         "counter traffic, which was measured at 64^3)")
    ap.add_argument("--stats-out", default=None, help="write per-step stats JSON here")
    ap.add_argument("--batch", action="store_true",
                    help="batched workload instead: 64 independent scenes through the serving engine")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload instead: Poisson time-step requests over 128 resident scenes")
    ap.add_argument("--eig", action="store_true",
                    help="eigen-projection microbenchmark on element Hessians harvested from the beam and the cube")
    ap.add_argument("--ablation", action="store_true",
                    help="paper variants instead: alpha/beta grid, PDN countdowns, mirroring (twisted beam)")
    ap.add_argument("--workers", type=int, default=8, help="engine worker threads (--batch / --serve)")
    ap.add_argument("--hw-queues", type=int, default=4,
                    help="--batch / --serve: HIP hardware queues of the process (at most 32; 4 measured "
                         "best: 2.7x over one worker on the batch, 1.5x with 8 queues, 1.1x with 16)")
    ap.add_argument("--requests", type=int, default=2000, help="--serve: number of requests")
    ap.add_argument("--no-pcg-batching", action="store_true",
                    help="--serve: solve each scene's systems in its own launches")
    ap.add_argument("--rate", type=float, default=200.0, help="--serve: mean arrival rate [1/s]")
    ap.add_argument("--launch-gaps", action="store_true",
                    help="only run the launch-cost probe (plain stream launches against HIP graph replays)")
    ap.add_argument("--read-bw-mib", type=int, default=0,
                    help="run the plain streaming read (csrc/probes/read_bw.hip) over this many MiB and exit")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run 5 plain device copies of this many MiB (HBM counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU layout is a design "
              "note, not a measured path", file=sys.stderr)
        sys.exit(2)
    if a.read_bw_mib:
        # HBM read rate of a plain streaming kernel over a resident buffer
        exe = os.path.join(ROOT, "paper_2505_21013_amd", "read_bw")
        if not os.path.exists(exe):
            sys.exit(f"{exe} is not built (python -c 'import __graft_entry__ as g; g.build()')")
        sys.exit(subprocess.run([exe, str(a.read_bw_mib)]).returncode)
    if a.launch_gaps:
        # 12 and 5 us: the product and the update of one PCG iteration on the twisted beam
        exe = os.path.join(ROOT, "paper_2505_21013_amd", "launch_gaps")
        if not os.path.exists(exe):
            sys.exit(f"{exe} is not built (python -c 'import __graft_entry__ as g; g.build()')")
        sys.exit(subprocess.run([exe, "12", "5"]).returncode)
    if a.ablation:
        print(json.dumps(run_ablation(a)), flush=True)
        return
    if a.eig:
        print(json.dumps(run_eig(a)), flush=True)
        return
    if a.batch or a.serve:
        # HIP reads this at initialisation
        os.environ["GPU_MAX_HW_QUEUES"] = str(max(1, min(32, a.hw_queues)))
        print(json.dumps(run_batch(a) if a.batch else run_serve(a)), flush=True)
        return

    import numpy as np
    import torch

    if a.calibrate_copy_mib:
        n = a.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": 5}))
        return

    torch.cuda.set_device(0)
    headline = "mixed" if a.precision == "mixed" else "fp64"
    runs = {headline: run_form(a, headline, torch, np)}
    if a.precision == "both":
        runs["mixed"] = run_form(a, "mixed", torch, np)
    R = runs[headline]
    K, info, tot, stats = a.steps, R["info"], R["tot"], R["stats"]
    out = {
        "metric": ("Newton time steps/s (PPN, %s) + 12x12 eigen-projections/s; p50/p99 step latency (1 GPU)"
                   % ("FP64" if headline == "fp64" else "mixed FP32/FP64")),
        "value": K / R["elapsed"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": a.warmup,
        "ms_per_step": R["elapsed"] / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if headline == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": (f"cube {a.cells or 64}^3 cells -> {info['n_tets']} tets / {info['n_verts']} verts, "
                                f"SNH E log-uniform [1e4,1e6] Pa, nu 0.48, dt 1/30 s, top pushed down "
                                f"60% over 50 steps; steps 1..{K}; mode {a.mode}"
                                if a.config == 2 else f"configuration {a.config}, mode {a.mode}"),
                   "mode": a.mode, "precision": headline, "n_tets": info["n_tets"],
                   "n_verts": info["n_verts"], "n_blocks": info["n_blocks"],
                   "parallelism": "single GPU"},
    }
    if form_params(a):
        out["config"]["params"] = form_params(a)
    out.update(summary(R, K, info, np))
    cfg = a.config if not a.cells else None
    out["roofline"] = roofline(R, headline, info, cfg)
    out["composite_roofline"] = composite_roofline(R, headline, info, K)
    if "mixed" in runs and headline == "fp64":
        M = runs["mixed"]
        diag = float(np.linalg.norm(M["X"].max(0) - M["X"].min(0)))
        m = {"value": K / M["elapsed"], "unit": "steps/s", "ms_per_step": M["elapsed"] / K * 1e3,
             "speedup_vs_fp64": (K / M["elapsed"]) / out["value"],
             "dtype": "f32+f64"}
        m.update(summary(M, K, info, np))
        m["refine_rounds_per_solve"] = M["tot"]["refine_rounds"] / max(M["tot"]["solves"], 1)
        m["max_position_diff_vs_fp64_run"] = float(np.max(np.abs(M["x"] - R["x"]))) / diag
        m["roofline"] = roofline(M, "mixed", info, cfg)
        m["composite_roofline"] = composite_roofline(M, "mixed", info, K)
        out["mixed"] = m
    if a.stats_out:
        with open(a.stats_out, "w") as f:
            json.dump(stats, f)
    if not a.no_cpu_baseline and not a.cells:
        tot = R["tot"]
        counts = {"newton_iters": tot["newton_iters"] / K, "pcg_iters": tot["pcg_iters"] / K,
                  "projected": tot["projected"] / K,
                  "ls_trials": (tot["newton_iters"] + tot["ls_backtracks"]) / K}
        out["cpu_baseline"] = cpu_baseline(a.config, counts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
