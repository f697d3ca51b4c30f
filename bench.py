"""Benchmark: RK4 steps/s on one large Fock sector, one MI355X.

Workload (one large sector): M = 8 modes on a periodic momentum grid,
omega_k = k^2/2, long-range V = 1/q^2 (zero transfer removed), Lambda = 0.02,
number eigenstate of seeded random occupations with N = 48 bosons in the
P = 0 sector (25,366,335 states), complex FP64 RK4 with dt = 5e-4, moments
every 50 steps.  One step = four fused H psi stage launches (plus the moment
reductions every 50th step).

    python bench.py [--gpus 1] [--steps 2000] [--warmup 20]

Prints one JSON line.  The CPU oracle is timed on a bounded sample of rows of
the same sector (see "cpu_baseline").
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# Vector-memory (texture) path: 256 CUs, 64 B per clock each into the vector
# L1, 2.4 GHz.  A 64-lane b128 gather (16 B per lane) occupies it for 16
# clocks, so this is also the gather-issue ceiling of the stage kernel.
CU_COUNT, CLOCK_GHZ, L1_BYTES_PER_CLK = 256, 2.4, 64
PEAK_GATHER_GBS = CU_COUNT * L1_BYTES_PER_CLK * CLOCK_GHZ
# Algorithmic bytes per state of the four fused stages (complex128 = 16 B):
#   stage 1: read psi, write acc and y2               = 48
#   stage 2: read y2, psi, acc; write acc and y3      = 80
#   stage 3: read y3, psi, acc; write acc and y4      = 80
#   stage 4: read y4, acc; write psi                  = 48
# Neighbour gathers re-read vectors already counted (ideal cache reuse).
STAGE_BYTES_PER_STATE = (48 + 80 + 80 + 48) / 4.0
KERNEL_SRC = os.path.join(ROOT, "paper_2111_00050_amd", "csrc", "fh_device.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_M8_N48_traffic.json")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(states: int, launch: dict):
    """HBM bytes per stage launch from committed rocprofv3 PMC counters, if
    they were taken on the current kernel source with the same launch
    schedule."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash() or t.get("states") != states:
        return None
    keys = ("blocks_per_cu", "xcd_order", "tile_order", "prefix_modes")
    if any(t.get("launch", {}).get(k) != launch.get(k) for k in keys):
        return None
    return t.get("bytes_per_launch")


def _oracle_rows_worker(job):
    """One CPU-baseline worker (a fresh interpreter, started before any GPU
    work): builds the oracle for the sector and times its gather-form H psi on
    a seeded sample of rows.  Returns (rows, seconds)."""
    import numpy as np

    import workloads as W
    from oracle import Oracle

    seed, nrows = job
    w = W.large_sector()
    orc = Oracle(w.M, w.pmod, w.omega, w.Lambda, w.V, w.sectors)
    psi = np.zeros(orc.total, np.complex128)
    rows = np.sort(np.random.default_rng(seed).choice(orc.total, size=nrows, replace=False))
    t0 = time.perf_counter()
    orc.apply_h_rows(psi, rows)
    return nrows, time.perf_counter() - t0


def adjoint_checkpoints(torch, nsteps: int, vec_bytes: int, frac: float = 0.8):
    """Checkpoint interval for fh_adjoint_rk4 that uses the free device memory.
    With kept stage inputs the last segment (a whole one: the first takes the
    remainder) is kept from the forward sweep and every other segment is
    recomputed once, so the recompute is nsteps - C steps: take the largest C
    whose work buffer (segments + 4C + 10 state vectors) fits in frac of what is
    free; else the largest C with recomputed stage inputs (segments + C + 10).
    Returns (C, kept)."""
    torch.cuda.empty_cache()  # blocks cached by torch count as free here
    free, _ = torch.cuda.mem_get_info()
    budget = frac * free
    for C in range(nsteps, 0, -1):
        if (-(-nsteps // C) + 4 * C + 10) * vec_bytes <= budget:
            return C, True
    for C in range(nsteps, 0, -1):
        if (-(-nsteps // C) + C + 10) * vec_bytes <= budget:
            return C, False
    return 1, False


def gathers_per_row(M: int) -> int:
    """Neighbour gathers the stage kernel issues per row: for each momentum
    class c of unordered pairs {i <= j} (class (i + j) mod M) with S_c pairs,
    S_c (S_c - 1) ordered (row pair, source pair) combinations."""
    cls = [0] * M
    for i in range(M):
        for j in range(i, M):
            cls[(i + j) % M] += 1
    return sum(c * (c - 1) for c in cls)


def apply_timing(fh, torch, model, basis, x, warmup=3, runs=20):
    """Median duration (s) of one H psi launch (fh_apply_h, APPLY mode) from
    HIP events recorded on the launch stream around each call."""
    out = torch.empty_like(x)
    for _ in range(warmup):
        fh.apply_h(model, basis, x, out)
    ts = []
    for _ in range(runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fh.apply_h(model, basis, x, out)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def copy_bandwidth(torch, nbytes=1 << 31, runs=10):
    """Device-to-device copy rate (read + write bytes / s, median of runs): the
    practical HBM peak on this GPU."""
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    ts.sort()
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / ts[len(ts) // 2] / 1e9


def apply_only(fh, torch, which: str, launches: int) -> dict:
    """H psi (APPLY) launches alone on one workload, for profiling: the one
    large sector (one column), or the field-number draws (M = 10, N = 30, all
    10 P) with one column (draw 0) or all 16 draws as one vector.  Default
    launch schedule of the basis.  Returns per-launch milliseconds (HIP events
    on the launch stream) after one warm-up launch."""
    import workloads as W

    w = W.large_sector() if which == "one_large_sector" else W.fieldnumber_draws(16, 30)
    model, basis = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, w.sectors)
    if w.init == "number":
        x, nrhs = fh.init_number(basis, w.init_params), 1
    else:
        nrhs = 16 if which == "fieldnumber_16" else 1
        x = fh.init_fieldnumber(basis, w.init_params if nrhs > 1 else w.init_params[0])
    print(f"[bench] apply-only {which}: {basis.total} states x {nrhs}", file=sys.stderr, flush=True)
    out = torch.empty_like(x)
    fh.apply_h(model, basis, x, out)
    ms = []
    for _ in range(launches):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fh.apply_h(model, basis, x, out)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    med = sorted(ms)[len(ms) // 2]
    return {"apply_only": which, "states": basis.total, "rhs": nrhs, "launch_ms": ms, "median_ms": med,
            "ns_per_row_column": med * 1e6 / (basis.total * nrhs)}


def host_info() -> dict:
    """nproc and the CPU model of this host (for the CPU-baseline line)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_workers() -> int:
    """Host cores for the CPU baseline: the process's CPU set, at most 16 (a
    one-GPU share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, target_s: float = 10.0):
    """Time the CPU oracle's gather-form H psi on samples of rows of the same
    sector, one thread and then one process per host core, and convert to RK4
    steps/s (4 H psi per step; the vector updates are negligible next to
    them).  Call before the GPU is touched: the workers are spawned."""
    import multiprocessing as mp

    import numpy as np

    from oracle import Oracle

    orc = Oracle(w.M, w.pmod, w.omega, w.Lambda, w.V, w.sectors)
    D = orc.total
    psi = np.zeros(D, np.complex128)
    rng = np.random.default_rng(77)
    rows = np.sort(rng.choice(D, size=200, replace=False))
    t0 = time.perf_counter()
    orc.apply_h_rows(psi, rows)
    per_row = (time.perf_counter() - t0) / len(rows)
    n = int(max(200, min(D, target_s / max(per_row, 1e-9))))
    rows = np.sort(rng.choice(D, size=n, replace=False))
    t0 = time.perf_counter()
    orc.apply_h_rows(psi, rows)
    dt1 = time.perf_counter() - t0
    one = 1.0 / (4.0 * D * dt1 / n)
    del orc, psi
    cores = cpu_workers()
    if cores == 1:
        return {"value": one, "unit": "RK4 steps/s", "cores": 1, "kind": "oracle", **host_info(),
                "sample": f"oracle gather-form H psi on {n} random rows of the {D}-state sector ({dt1:.1f} s), "
                          f"scaled to 4 H psi per RK4 step"}
    with mp.get_context("spawn").Pool(cores) as pool:
        out = pool.map(_oracle_rows_worker, [(1000 + i, n) for i in range(cores)])
    rows_all = sum(r for r, _ in out)
    wall = max(t for _, t in out)
    return {
        "value": 1.0 / (4.0 * D * wall / rows_all),
        "unit": "RK4 steps/s",
        "cores": cores,
        "kind": "oracle",
        **host_info(),
        "one_thread_value": one,
        "sample": f"oracle gather-form H psi, {cores} processes on independently seeded samples of {n} random rows of "
                  f"the {D}-state sector each ({wall:.1f} s of parallel time), scaled to 4 H psi per RK4 step; "
                  f"one thread: {one:.3g} steps/s",
    }


def forms():
    """The three forms of the path next to their plain counterparts, each on
    its own workload at full size with a bounded number of steps:
      batched   : one persistent launch per stage over all sectors, the step
                  captured in a HIP graph, vs one launch per sector per stage
                  (M=6 coherent state, mean 40 bosons, 541 sectors; and the
                  paper's M=5 long-range coherent problem at r = 4, 176
                  non-empty sectors of at most 16,451 states);
      multi_rhs : 16 field-number phase draws as one 16-column vector vs the
                  same draws run one at a time (M=10, N=30, all 10 P);
      adjoint   : forward + discrete adjoint (gradients of J), and the
                  forward-mode tangent in Lambda, vs the forward
                  alone (M=6 number state N=30, 3000 steps; M=6 coherent
                  state, mean 20, 331 sectors, 100 steps; one M=10 field-number
                  draw, 212M states, 10 steps), with a central difference of
                  J in Lambda on the first.
      chebyshev : the Chebyshev propagator (exp(-i H dt) to 1e-14 per step, steps
                  of 0.05) vs RK4 at the bench's dt = 5e-4 over t = 0.2 on the
                  bench's sector; their difference is RK4's truncation error.
    Equal-accuracy check: the two paths of a pair return the same amplitudes
    (max |difference| is reported; the kernels sum in the same order)."""
    import numpy as np
    import torch

    import paper_2111_00050_amd as fh
    import workloads as W

    sync = torch.cuda.synchronize
    c128 = torch.complex128

    def log(msg):
        print(f"[bench/forms] {msg}", file=sys.stderr, flush=True)

    def timed(fn):
        sync()
        t0 = time.perf_counter()
        r = fn()
        sync()
        return r, time.perf_counter() - t0

    out = {}
    # ---- batched vs per sector
    w = W.batched_coherent()
    model, basis = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, w.sectors)
    D = basis.total
    log(f"batched: {D} states in {len(w.sectors)} sectors")
    psi0 = fh.init_coherent(basis, w.init_params)
    work = torch.empty(3 * D, dtype=c128, device="cuda")
    steps, fin, sps = 3, {}, {}
    stream = torch.cuda.Stream()  # graph capture needs a non-default stream
    for name, flags in (("batched", fh.FH_GRAPH), ("per_sector", fh.FH_PER_SECTOR)):
        psi = psi0.clone()
        sync()
        with torch.cuda.stream(stream):
            fh.evolve_rk4(model, basis, psi, w.dt, 1, flags=flags, work=work)
            _, t = timed(lambda: fh.evolve_rk4(model, basis, psi, w.dt, steps, flags=flags, work=work))
        sps[name], fin[name] = steps / t, psi
        log(f"  {name}: {steps / t:.3f} steps/s")
    out["batched"] = {
        "workload": "M=6 coherent, mean 40 bosons, N 0..90 x all P, contact V, Lambda=0.05, dt=1e-3",
        "states": D, "sectors": sum(1 for d in basis.dims if d > 0), "timed_steps": steps,
        "steps_per_s": sps["batched"], "per_sector_steps_per_s": sps["per_sector"],
        "speedup": sps["batched"] / sps["per_sector"],
        "max_abs_diff": float((fin["batched"] - fin["per_sector"]).abs().max()),
    }
    del psi0, psi, work, fin
    model.close()
    basis.close()
    torch.cuda.empty_cache()

    # ---- batched vs per sector on many small sectors (the paper's own size)
    w = W.paper_problem("coherent", "longrange", 4)
    sectors = W.all_sectors(w.M, 35)  # Poisson(20) weight >= 0.999
    model, basis = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, sectors)
    D = basis.total
    log(f"batched (small sectors): {D} states in {len(sectors)} sectors")
    psi0 = fh.init_coherent(basis, w.init_params[0])
    work = torch.empty(3 * D, dtype=c128, device="cuda")
    steps, fin, sps = 200, {}, {}
    for name, flags in (("batched", fh.FH_GRAPH), ("per_sector", fh.FH_PER_SECTOR)):
        psi = psi0.clone()
        sync()
        with torch.cuda.stream(stream):
            fh.evolve_rk4(model, basis, psi, 1e-3, 2, flags=flags, work=work)
            _, t = timed(lambda: fh.evolve_rk4(model, basis, psi, 1e-3, steps, flags=flags, work=work))
        sps[name], fin[name] = steps / t, psi
        log(f"  {name}: {steps / t:.1f} steps/s")
    out["batched_small"] = {
        "workload": "M=5 coherent, mean 20 bosons (the paper's long-range problem, r = 4, exact momentum), "
                    "N 0..35 x all P, dt=1e-3",
        "states": D, "sectors": sum(1 for d in basis.dims if d > 0), "timed_steps": steps,
        "steps_per_s": sps["batched"], "per_sector_steps_per_s": sps["per_sector"],
        "speedup": sps["batched"] / sps["per_sector"],
        "max_abs_diff": float((fin["batched"] - fin["per_sector"]).abs().max()),
    }
    del psi0, psi, work, fin
    model.close()
    basis.close()
    torch.cuda.empty_cache()

    # ---- 16 columns vs 16 single runs
    w = W.fieldnumber_draws(16, 30)
    model, basis = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, w.sectors)
    D = basis.total
    log(f"multi-rhs: {D} states x 16 draws")
    steps = 2
    psi = fh.init_fieldnumber(basis, w.init_params)
    work = torch.empty(3 * D * 16, dtype=c128, device="cuda")
    fh.evolve_rk4(model, basis, psi, w.dt, 1, work=work)
    _, tm = timed(lambda: fh.evolve_rk4(model, basis, psi, w.dt, steps, work=work))
    col0 = psi[:, 0].clone()
    del psi, work
    torch.cuda.empty_cache()
    log(f"  16 columns: {steps / tm:.4f} steps/s")
    psi1 = fh.init_fieldnumber(basis, w.init_params[0])
    work1 = torch.empty(3 * D, dtype=c128, device="cuda")
    fh.evolve_rk4(model, basis, psi1, w.dt, 1, work=work1)
    _, ts = timed(lambda: fh.evolve_rk4(model, basis, psi1, w.dt, steps, work=work1))
    log(f"  one column: {steps / ts:.4f} steps/s")
    out["multi_rhs"] = {
        "workload": "M=10 field-number states, 16 phase draws, N=30 x all 10 P, contact V, Lambda=0.01, dt=2e-4",
        "states": D, "rhs": 16, "timed_steps": steps,
        "steps_per_s_16_draws": steps / tm, "steps_per_s_16_draws_one_at_a_time": steps / ts / 16,
        "speedup": 16 * ts / tm,
        "max_abs_diff_draw0": float((psi1 - col0).abs().max()),
    }
    del psi1, work1, col0
    model.close()
    basis.close()
    torch.cuda.empty_cache()

    # ---- Chebyshev propagator vs RK4 over the same simulated time
    w = W.large_sector()
    model, basis = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, w.sectors)
    log(f"chebyshev: {w.name}, {basis.total} states")
    T, cdt = 0.2, 0.05
    psi0 = fh.init_number(basis, w.init_params)
    p_r = psi0.clone()
    _, t_rk4 = timed(lambda: fh.evolve_rk4(model, basis, p_r, w.dt, int(round(T / w.dt))))
    rho, t_rho = timed(lambda: fh.spectral_radius(model, basis, iters=60))
    R = 1.1 * rho + 1e-9
    p_c = psi0.clone()
    _, t_ch = timed(lambda: fh.evolve_chebyshev(model, basis, p_c, cdt, int(round(T / cdt)), -R, R))
    p_h = psi0.clone()
    fh.evolve_chebyshev(model, basis, p_h, cdt / 2, int(round(2 * T / cdt)), -R, R)
    nrm = float(torch.linalg.vector_norm(p_h))
    out["chebyshev"] = {
        "workload": w.name + f", evolved to t = {T}",
        "states": basis.total, "rk4_dt": w.dt, "chebyshev_dt": cdt, "spectral_interval": [-R, R],
        "rk4_s": t_rk4, "chebyshev_s": t_ch, "spectral_radius_s": t_rho, "speedup": t_rk4 / (t_ch + t_rho),
        "terms_per_step": int(len(fh.chebyshev_coefficients(R * cdt))),
        "rel_diff_rk4_vs_chebyshev": float(torch.linalg.vector_norm(p_r - p_c)) / nrm,
        "rel_diff_chebyshev_step_halved": float(torch.linalg.vector_norm(p_c - p_h)) / nrm,
    }
    log(f"  rk4 {t_rk4:.2f} s, chebyshev {t_ch:.2f} s + bound {t_rho:.2f} s")
    del psi0, p_r, p_c, p_h
    model.close()
    basis.close()
    torch.cuda.empty_cache()

    # ---- adjoint vs forward
    adj = []
    for w, obj, steps, nd in ((W.adjoint_number(30), fh.FH_J_NMODE, 3000, 1),
                              (W.adjoint_coherent(20.0), fh.FH_J_Q, 100, 1),
                              (W.fieldnumber_draws(16, 30), fh.FH_J_PO, 10, 1),
                              (W.fieldnumber_draws(16, 30), fh.FH_J_PO, 10, 2)):
        model, basis = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, w.sectors)
        log(f"adjoint: {w.name}, {basis.total} states x {nd}, {steps} steps")

        def init(b=basis, w=w, nd=nd):
            if w.init == "number":
                return fh.init_number(b, w.init_params)
            if w.init == "fieldnumber":
                return fh.init_fieldnumber(b, w.init_params[0] if nd == 1 else w.init_params[:nd])
            return fh.init_coherent(b, w.init_params)

        ck, keep = adjoint_checkpoints(torch, steps, 16 * basis.total * nd)
        # work buffers are allocated outside the timed calls (both sides)
        psi = init()
        fwork = torch.empty(3 * basis.total * nd, dtype=c128, device="cuda")
        _, tf = timed(lambda: fh.evolve_rk4(model, basis, psi, w.dt, steps, work=fwork))
        del psi, fwork
        psi0 = init()
        size_fn = fh._lib.fh_adjoint_work_states_kept if keep else fh._lib.fh_adjoint_work_states
        awork = torch.empty(int(size_fn(steps, ck)) * basis.total * nd, dtype=c128, device="cuda")
        res, ta = timed(lambda: fh.adjoint_rk4(model, basis, psi0, w.dt, steps, ck, obj, 0, work=awork))
        name = w.name + ((", draw 0 only" if nd == 1 else f", draws 0..{nd - 1} in one vector")
                         if w.init == "fieldnumber" else "")
        rec = {"workload": name, "states": basis.total, "columns": nd, "steps": steps, "checkpoint_every": ck,
               "stage_inputs_kept": keep,
               "objective": {fh.FH_J_Q: "Q", fh.FH_J_NMODE: "<n_0>(T)", fh.FH_J_PO: "1 - lambda_p/n_tot"}[obj],
               "forward_s": tf, "adjoint_s": ta, "ratio": ta / tf,
               "J": [float(x) for x in res["J"]], "dJ_dLambda": [float(x) for x in res["dLambda"]]}
        if nd > 1:
            # per-draw time against the same draws adjointed one at a time
            lam_both = res["lambda0"]
            res1, ta1 = None, 0.0
            diffs = []
            del awork
            ck1, keep1 = adjoint_checkpoints(torch, steps, 16 * basis.total)
            size_fn = fh._lib.fh_adjoint_work_states_kept if keep1 else fh._lib.fh_adjoint_work_states
            awork = torch.empty(int(size_fn(steps, ck1)) * basis.total, dtype=c128, device="cuda")
            for q in range(nd):
                p1 = fh.init_fieldnumber(basis, w.init_params[q])
                r1, t1 = timed(lambda: fh.adjoint_rk4(model, basis, p1, w.dt, steps, ck1, obj, 0, work=awork))
                ta1 += t1
                diffs.append(max(abs(float(r1["dLambda"][0]) - float(res["dLambda"][q])),
                                 float(np.abs(r1["dV"][0] - res["dV"][q]).max()),
                                 float((r1["lambda0"][:, 0] if r1["lambda0"].dim() > 1 else r1["lambda0"]).sub(
                                     lam_both[:, q]).abs().max())))
                del p1, r1
            rec.update({"one_at_a_time_checkpoint_every": ck1, "one_at_a_time_adjoint_s": ta1,
                        "per_draw_s": ta / nd, "per_draw_one_at_a_time_s": ta1 / nd,
                        "speedup_over_one_at_a_time": ta1 / ta, "max_abs_diff_vs_one_at_a_time": max(diffs)})
            del lam_both
        else:
            tan, tt = timed(lambda: fh.tangent_rk4(model, basis, psi0, w.dt, steps, obj, 0))
            del tan["psi"], tan["dpsi"]
            rec.update({"tangent_s": tt, "tangent_ratio": tt / tf, "tangent_dJ_dLambda": float(tan["dLambda"][0])})
        if steps == 3000:
            h = 1e-6
            Jpm = []
            for sgn in (1, -1):
                mh = fh.Model(w.M, w.omega, w.Lambda + sgn * h, w.V)
                Jpm.append(float(fh.adjoint_rk4(mh, basis, init(), w.dt, steps, ck, obj, 0, work=awork)["J"][0]))
                mh.close()
            fd = (Jpm[0] - Jpm[1]) / (2 * h)
            rec["dJ_dLambda_central_difference"] = fd
        log(f"  adjoint ratio {ta / tf:.2f} (checkpoint every {ck}, kept {keep})")
        adj.append(rec)
        del psi0, res, awork
        model.close()
        basis.close()
        torch.cuda.empty_cache()
    out["adjoint"] = adj
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched / multi-rhs / adjoint comparisons")
    ap.add_argument("--forms-only", action="store_true", help="run only the form comparisons (one JSON object)")
    ap.add_argument("--apply-only", choices=["one_large_sector", "fieldnumber_1", "fieldnumber_16"], default=None,
                    help="only time --launches H psi launches (APPLY) on this workload (for profilers)")
    ap.add_argument("--launches", type=int, default=3)
    ap.add_argument("--autotune", action="store_true",
                    help="let fh_basis_autotune pick the launch schedule instead of the next four options")
    ap.add_argument("--no-autotune", action="store_true", help="(the default) use the next four options")
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--xcd-order", type=int, default=3)
    ap.add_argument("--tile-order", type=int, default=0)
    ap.add_argument("--prefix-modes", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); "
              "the sector evolution is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import workloads as W

    cpu = None
    if not args.no_cpu_baseline and not args.forms_only:
        # before any GPU work, so that the worker processes start from a clean process
        print("[bench] timing the CPU oracle on samples", file=sys.stderr, flush=True)
        cpu = cpu_baseline(W.large_sector())

    import numpy as np
    import torch

    import paper_2111_00050_amd as fh

    torch.cuda.set_device(0)
    if args.apply_only:
        print(json.dumps(apply_only(fh, torch, args.apply_only, args.launches)), flush=True)
        return
    if args.forms_only:
        print(json.dumps({"forms": forms()}), flush=True)
        return
    w = W.large_sector()
    model = fh.Model(w.M, w.omega, w.Lambda, w.V)
    basis = fh.Basis(w.M, w.sectors)
    D = basis.total
    psi = fh.init_number(basis, w.init_params)
    if not args.autotune:
        # the given schedule (default: every workgroup the CU holds, per-XCD
        # tile queues over chunks dealt to the XCDs in turn, plain 256-row tiles)
        basis.set_launch(args.blocks_per_cu, args.xcd_order)
        basis.set_tile_order(args.tile_order, args.prefix_modes)
        launch = {"blocks_per_cu": args.blocks_per_cu, "xcd_order": args.xcd_order,
                  "tile_order": args.tile_order, "prefix_modes": args.prefix_modes, "autotuned": False}
    else:
        # untimed: pick the launch schedule of the stage kernel for this basis
        launch, _ = fh.autotune(model, basis, psi)
        launch["autotuned"] = True
        print(f"[bench] autotuned launch {launch}", file=sys.stderr, flush=True)
    work = torch.empty(3 * D, dtype=torch.complex128, device="cuda")
    print(f"[bench] {w.name}: {D} states; warmup {args.warmup} steps", file=sys.stderr, flush=True)
    if args.warmup > 0:
        fh.evolve_rk4(model, basis, psi, w.dt, args.warmup, work=work)
    torch.cuda.synchronize()
    # Moments every 50 steps as the workload asks, from step 0 on, all inside
    # the timed region.  When the timed steps are not a multiple of 50, step 0
    # is the only such step: its moments are timed on their own and the run
    # records none; the drift checks compare them with the last state's
    # moments, taken after the timed region (not a step of the cadence).
    every = w.every if args.steps % w.every == 0 else 0
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    rec0 = None if every else fh.moments(basis, psi)
    res = fh.evolve_rk4(model, basis, psi, w.dt, args.steps, every=every, flags=fh.FH_TIMING, work=work)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps_per_s = args.steps / elapsed
    avg_stage_s = res.stage_ms / 1e3 / max(1, res.stage_launches)
    alg_bytes = STAGE_BYTES_PER_STATE * D
    achieved = alg_bytes / avg_stage_s / 1e9
    traffic = measured_traffic(D, launch)
    if every:
        first, last = fh.unpack_moments(w.M, res.records[0, 0]), fh.unpack_moments(w.M, res.records[-1, 0])
        rec_steps = [int(x) for x in res.steps]
    else:
        first, last = rec0, fh.moments(basis, psi)
        rec_steps = [0, args.steps]
    norms = (first[0], last[0])
    obs0 = fh.derive(w.M, *first)
    obsT = fh.derive(w.M, *last)
    # after the timed region: H psi launches timed on their own, and the
    # device's copy bandwidth (the practical peak)
    print("[bench] timing H psi launches and a device copy", file=sys.stderr, flush=True)
    apply_s = apply_timing(fh, torch, model, basis, psi)
    copy_gbs = copy_bandwidth(torch)
    gpr = gathers_per_row(w.M)
    gather_gbs = gpr * 16.0 * D / avg_stage_s / 1e9
    line = {
        "metric": "RK4 Fock steps/s",
        "value": steps_per_s,
        "unit": "RK4 steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "one large sector: M=8, N=48, P=0 (25,366,335 states), w=k^2/2, long-range V, "
                        "Lambda=0.02, number eigenstate (seeded), complex FP64 RK4 dt=5e-4, moments every 50 steps",
            "states": D,
            "parallelism": "single GPU",
        },
        "hpsi_per_s": 1.0 / apply_s,
        "hpsi_ms": 1e3 * apply_s,
        "hpsi_timing": "median of 20 fh_apply_h launches (APPLY mode, 3 warm-up) between HIP events on the launch "
                       "stream, after the timed steps",
        "launch": launch,
        "stage_kernel_ms": 1e3 * avg_stage_s,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "bytes_model": f"{STAGE_BYTES_PER_STATE:.0f} B per state per stage launch (mean over the four fused "
                           "stages: 48, 80, 80, 48 B; every vector once, the gathered vector once)",
            "practical_peak": copy_gbs,
            "frac_of_practical_peak": achieved / copy_gbs,
            "traffic_frac": (None if traffic is None else traffic / avg_stage_s / 1e9 / PEAK_HBM_GBS),
            "binding_unit": "vector-memory gather path (texture addresser / L1, waiting on L2 misses); see "
                            "roofline_gather",
        },
        "roofline_gather": {
            "bound": "vector-memory gather issue",
            "gathers_per_row": gpr,
            "achieved": gather_gbs,
            "peak": PEAK_GATHER_GBS,
            "unit": "GB/s",
            "frac": gather_gbs / PEAK_GATHER_GBS,
            "model": f"{gpr} b128 neighbour gathers (16 B per lane) per row per stage launch; peak {CU_COUNT} CUs x "
                     f"{L1_BYTES_PER_CLK} B/clock x {CLOCK_GHZ} GHz into the vector L1",
        },
        "checks": {
            "records_at_steps": rec_steps,
            "norm_drift": float(abs(norms[-1] - norms[0])),
            "n_tot_drift": float(abs(obsT["n_tot"] - obs0["n_tot"])),
            "lambda_p_end": obsT["lambda_p"],
        },
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    if not args.no_forms:
        del psi, work
        model.close()
        basis.close()
        torch.cuda.empty_cache()
        line["forms"] = forms()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
