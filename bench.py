"""Benchmark: cache-blocked gate application on one MI355X.

Workload: the Quantum-Volume-style circuit at 33 qubits, complex128, in place
(a 128 GiB state): depth 33, each layer a seeded random qubit permutation
paired into Haar SU(4) gates (528 gates), seed 0.  One step applies the whole
circuit through the blocked path (one kernel per section, every section one
HBM read + one write of the state).  The per-gate path (one kernel per gate)
runs once on the same circuit for the speedup and the parity check
(1 - F between the two results, FP64 overlap on the device).

Prints one JSON line.  `value` = algorithmic bytes of the blocked path
(2 * 2^n * 16 B per section) / timed wall time, in GB/s.
"""

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X vector peaks (256 CUs x 2.4 GHz): FP64 78.6 TFLOP/s; FP32 157.3 TFLOP/s,
# of which single-issue (non-packed) FP32 reaches half
ALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
# sections timed per autotune candidate (scaled by the candidate's section count),
# then the best TUNE_REFINE estimates timed on whole applies
TUNE_SECTIONS = 6
TUNE_REFINE = 3
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "section_kernel_qv33_c128_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None,
                    help="qubits (default 33; 32 for the host workload, whose state must fit "
                         "the pinned host memory a process may allocate)")
    ap.add_argument("--dtype", choices=["c128", "c64"], default="c128")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--skip-pergate", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--chunk-bits", type=int, default=None)
    ap.add_argument("--pinned", type=int, default=None)
    ap.add_argument("--fusion", type=int, default=None)
    ap.add_argument("--register-bits", type=int, default=None)
    ap.add_argument("--io-phases", type=int, default=None)
    ap.add_argument("--section-kernel", type=int, default=None,
                    help="0: register-phase kernel, 1: LDS-resident chunk, 2: paired register "
                         "phases, 3: LDS-resident chunk with fused 4-5 qubit blocks on MFMA")
    ap.add_argument("--planner", type=int, default=None,
                    help="0 default, 1 greedy, 2 beam search, 3 exact (small circuits)")
    ap.add_argument("--autotune", choices=["live", "cache", "off"], default="live",
                    help="live: tune on this workload now (the default); cache: reuse a stored "
                         "result for the same (arch, dtype, n, circuit) if there is one; off: "
                         "library defaults.  Explicit plan options also turn it off.")
    ap.add_argument("--tune-cache", default=None,
                    help="autotune cache file (default: $QSV_AUTOTUNE_CACHE or ~/.cache/qsv)")
    ap.add_argument("--hbm-budget-gib", type=float, default=48.0,
                    help="host workload: device memory for the slice buffers")
    ap.add_argument("--sections", type=int, default=3,
                    help="host workload: sections timed per step")
    ap.add_argument("--workload", choices=["qv", "trajectories", "adjoint", "host", "density"],
                    default="qv",
                    help="qv: the headline blocked apply (default); trajectories: 512 noisy "
                         "trajectories in one graph launch; adjoint: 20-qubit ansatz gradients; "
                         "host: state in pinned host memory; density: noisy 16-qubit density "
                         "matrix")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("section_core.hpp", "section_kernels.hpp", "section_kernel.hip", "section_c128.hip",
              "section_c64.hip", "section_paired.hip", "section_lds.hip", "device.hpp",
              "qsv_internal.hpp", "planner.cpp"):
        with open(os.path.join(ROOT, "paper_2102_02957_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        return 1


def one_thread():
    """Context that limits BLAS/OpenMP pools to one thread (the oracle's
    elementwise NumPy work is single-threaded anyway), so `cores` is 1."""
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(1)
    except Exception:  # pragma: no cover
        import contextlib
        return contextlib.nullcontext()


def cpu_baseline(n_target, gates_target, blocked_bytes, seed):
    """The oracle as it stands, on one host core, on a bounded sample of the
    same workload: a 24-qubit Quantum-Volume circuit, gates applied until ~15 s
    have passed; the per-gate-per-amplitude time is scaled to the full circuit."""
    with one_thread():
        return _cpu_baseline(n_target, gates_target, blocked_bytes, seed)


def _cpu_baseline(n_target, gates_target, blocked_bytes, seed):
    import numpy as np
    import oracle
    from paper_2102_02957_amd import workloads as W
    threads = blas_threads()
    ns = 24
    gates = W.quantum_volume(ns, ns, seed)
    psi = oracle.zero_state(ns)
    t0 = time.perf_counter()
    done = 0
    for g in gates:
        oracle.apply_gate(psi, ns, g)
        done += 1
        if time.perf_counter() - t0 > 15.0:
            break
    dt = time.perf_counter() - t0
    per_gate_amp = dt / (done * float(1 << ns))
    t_full = per_gate_amp * len(gates_target) * float(1 << n_target)
    return {
        "value": blocked_bytes / t_full / 1e9,
        "unit": "GB/s",
        "cores": int(threads),
        "host_cores": len(os.sched_getaffinity(0)),
        "kind": "oracle",
        "sample": "NumPy oracle, %d of %d SU(4) gates of a %d-qubit QV circuit in %.1f s; "
                  "time per gate per amplitude scaled x%d gates x2^%d amplitudes "
                  "(extrapolated %.0f s for the %d-qubit circuit)"
                  % (done, len(gates), ns, dt, len(gates_target), n_target, t_full, n_target),
        "cpu": platform.processor() or platform.machine(),
        "affinity_cores": len(os.sched_getaffinity(0)),
    }


SECTION_KERNELS = {0: "registers", 1: "lds", 2: "paired", 3: "mfma"}


def section_kernel_name(kind, dt, B, r):
    t = "double" if dt == B.QSV_C128 else "float"
    return {1: "k_section_lds<%s, ...>" % t,
            2: "k_section_paired<%s>" % t,
            3: "k_section_lds<%s, 3, true> (MFMA blocks)" % t}.get(kind, "k_section<%s, %d, ...>" % (t, r))


def roofline(st, dt, B, steps, pass_bytes, achieved_gbs, avg_launch_ms, sec_ms, launches, traffic,
             kind=0):
    """The section kernel against both of its rooflines.  Per launch it moves one
    pass (2 * 2^n * es bytes) and performs section_flops / sections FP operations;
    the binding roofline is the one whose floor (work / peak) is longer."""
    fdt = "f64" if dt == B.QSV_C128 else "f32"
    alu_peak = ALU_PEAK_TFLOPS[fdt]
    flops_launch = st["section_flops"] / max(1, st["n_sections"])
    t_alu = flops_launch / (alu_peak * 1e12)
    t_hbm = pass_bytes / (HBM_PEAK_GBS * 1e9)
    alu_tflops = st["section_flops"] * steps / (sec_ms * 1e-3) / 1e12
    hbm = {"achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "floor_ms": round(t_hbm * 1e3, 2),
           "traffic": traffic}
    alu = {"achieved": round(alu_tflops, 2), "peak": alu_peak, "unit": "TFLOP/s",
           "frac": round(alu_tflops / alu_peak, 4), "floor_ms": round(t_alu * 1e3, 2),
           "dtype": fdt}
    main = alu if t_alu > t_hbm else hbm
    out = {"bound": "alu" if t_alu > t_hbm else "hbm"}
    out.update({k: main[k] for k in ("achieved", "peak", "unit", "frac")})
    out["traffic"] = traffic
    out.update({"kernel": section_kernel_name(kind, dt, B, st["register_bits"]) + " (one launch per section)",
                "avg_launch_ms": round(avg_launch_ms, 3), "launches": launches,
                "hbm": hbm, "alu": alu})
    return out


def gpu_arch(torch):
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # pragma: no cover
        return "unknown"


def autotune(args, torch, B, dtype, n, circuit_class, run):
    """Choose plan options with the library's autotuner.  run() -> (chosen,
    candidates, ms).  Returns (options dict or None, record for the JSON line)."""
    explicit = any(getattr(args, k) is not None for k in
                   ("chunk_bits", "pinned", "fusion", "register_bits", "io_phases",
                    "section_kernel", "planner"))
    if args.autotune == "off" or explicit:
        return None, {"mode": "off" if not explicit else "explicit options"}
    cache = B.AutotuneCache(args.tune_cache)
    key = B.AutotuneCache.key(gpu_arch(torch), dtype, n, circuit_class)
    t0 = time.perf_counter()
    if args.autotune == "live":
        chosen, cands, ms = run()
        cache.put(key, chosen, cands, ms)
        entry, hit = cache.get(key), False
    else:
        entry, hit = cache.tune(key, run)
    tune_s = time.perf_counter() - t0
    log("autotune %s: %s (%s, %.1f s)" % (key, entry["chosen"], "cache" if hit else "measured", tune_s))
    rec = {"mode": args.autotune, "key": key, "cache_hit": hit, "tune_s": round(tune_s, 2),
           "chosen": entry["chosen"],
           "candidates": [{"options": c, "ms": m} for c, m in zip(entry["candidates"], entry["ms"])]}
    return dict(entry["chosen"]), rec


def timed_calls(torch, fn, steps, warmup):
    """Run fn warmup + steps times on the current stream; return the wall time
    of the timed calls (seconds) and the event time on the current stream (ms)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, e0.elapsed_time(e1)


def bench_trajectories(args, torch, B, W):
    """512 Pauli-noise trajectories (10-20 qubits, depth 40, p = 1e-3),
    complex64 with FP64 renormalisation: one captured graph per call."""
    trajs = W.noisy_trajectories(512, 10, 20, 40, 1e-3, args.seed)
    offs, o = [], 0
    for n, _ in trajs:
        offs.append(o)
        o += 1 << n
    ctx = B.Context(B.QSV_C64)
    states = torch.empty(o, dtype=torch.complex64, device="cuda")

    def tune():
        cands = B.batch_candidates(B.QSV_C64)
        best, ms = ctx.autotune_batch(trajs, offs, states, candidates=cands, reps=2)
        return best, cands, ms

    chosen, tune_rec = autotune(args, torch, B, B.QSV_C64, 20, "512 noisy trajectories 10-20q "
                                "depth 40 seed %d" % args.seed, tune)
    opts = chosen or dict(chunk_bits=args.chunk_bits, pinned_low_bits=args.pinned,
                          fusion_max_qubits=args.fusion, register_bits=args.register_bits)
    t0 = time.perf_counter()
    plans = [B.Plan(n, g, B.QSV_C64, **opts) for n, g in trajs]
    t_plan = time.perf_counter() - t0
    norms = torch.empty(len(trajs), dtype=torch.float64, device="cuda")
    step_bytes = sum(p.stats()["n_sections"] * 2.0 * (1 << p.n) * 8 for p in plans)
    gates = sum(len(g) for _, g in trajs)
    wall, ev_ms = timed_calls(torch, lambda: ctx.batch_run(plans, offs, states, norms),
                              args.steps, max(1, args.warmup))
    nh = norms.cpu().numpy()
    log("trajectories: %.3f ms per launch, norms in [%.6f, %.6f]" % (ev_ms / args.steps, nh.min(), nh.max()))
    ms = wall * 1e3 / args.steps
    rec = {
        "metric": "noisy trajectories per second (512 states, 10-20 qubits, one graph launch)",
        "value": round(len(trajs) * args.steps / wall, 1), "unit": "trajectories/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512 trajectories, n ~ U{10..20}, depth 40 U3+CX, Pauli p=1e-3, "
                               "complex64, seed %d" % args.seed,
                   "gates": gates, "states_mib": round(o * 8 / 2 ** 20, 1), "plan_s": round(t_plan, 3),
                   "chunk_bits": max(p.stats()["chunk_bits"] for p in plans),
                   "register_bits": plans[0].stats()["register_bits"],
                   "fusion_max_qubits": plans[0].stats()["fusion_max_qubits"]},
        "gates_per_s": round(gates * args.steps / wall, 1),
        "roofline": {"bound": "hbm", "kernel": "batch graph (k_batch_init, k_batch_step per depth, k_batch_norms, k_batch_scale)",
                     "achieved": round(step_bytes / (ev_ms / args.steps * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(step_bytes / (ev_ms / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "note": "algorithmic bytes = sum over trajectories of sections x 2 x 2^n x 8 B; "
                             "states of 10-20 qubits are largely cache-resident"},
        "autotune": tune_rec,
    }
    if not args.skip_cpu:
        import oracle
        sample = sorted(range(len(trajs)), key=lambda b: trajs[b][0])
        t0 = time.perf_counter()
        work_done, k = 0.0, 0
        with one_thread():
            while k < len(sample) and time.perf_counter() - t0 < 10.0:
                n, g = trajs[sample[k]]
                oracle.apply_circuit(n, g)
                work_done += len(g) * float(1 << n)
                k += 1
        dt_cpu = time.perf_counter() - t0
        work_all = sum(len(g) * float(1 << n) for n, g in trajs)
        t_full = dt_cpu * work_all / work_done
        rec["cpu_baseline"] = {"value": round(len(trajs) / t_full, 3), "unit": "trajectories/s",
                               "cores": 1, "kind": "oracle", "host_cores": len(os.sched_getaffinity(0)),
                               "sample": "%d smallest trajectories in %.1f s, scaled by gates x amplitudes "
                                         "to all 512 (extrapolated %.0f s)" % (k, dt_cpu, t_full)}
    print(json.dumps(rec), flush=True)


def bench_adjoint(args, torch, B, W):
    """Adjoint gradient: 20-qubit hardware-efficient ansatz, 40 layers of RY.RZ
    + CX ring (1600 parameters), batch 64, H = sum Z_i Z_{i+1} (periodic)."""
    n, layers, batch = 20, 40, 64
    dt = B.QSV_C128 if args.dtype == "c128" else B.QSV_C64
    tdt = torch.complex128 if dt == B.QSV_C128 else torch.complex64
    es = 16 if dt == B.QSV_C128 else 8
    tmpl = W.hardware_efficient_ansatz(n, layers)
    theta = torch.from_numpy(W.ansatz_parameters(n, layers, batch, args.seed)).cuda()
    terms = [(1.0, (1 << i) | (1 << ((i + 1) % n))) for i in range(n)]
    ctx = B.Context(dt)
    psi = torch.empty(batch << n, dtype=tdt, device="cuda")
    lam = torch.empty_like(psi)

    def tune():
        cands = B.adjoint_candidates(dt, n)
        best, ms = ctx.autotune_adjoint(n, tmpl, terms, theta, psi, lam, candidates=cands, reps=1)
        return best, cands, ms

    chosen, tune_rec = autotune(args, torch, B, dt, n, "hardware-efficient ansatz 40 layers "
                                "batch %d seed %d" % (batch, args.seed), tune)
    # without tuning: chunk 11 with 8 amplitudes per thread (psi and lambda both sit
    # in registers during the reverse sweep; r = 3 keeps that kernel at 3 waves per SIMD)
    opts = chosen or dict(fusion_max_qubits=2,
                          chunk_bits=args.chunk_bits if args.chunk_bits is not None else 11,
                          register_bits=args.register_bits if args.register_bits is not None else 3,
                          pinned_low_bits=args.pinned)
    t0 = time.perf_counter()
    plan = B.Plan(n, tmpl, dt, **opts)
    t_plan = time.perf_counter() - t0
    S = plan.stats()["n_sections"]
    energy = torch.empty(batch, dtype=torch.float64, device="cuda")
    grad = torch.empty(batch, 2 * n * layers, dtype=torch.float64, device="cuda")
    call = lambda: ctx.adjoint_grad(plan, terms, theta, psi, lam, energy, grad)
    wall, ev_ms = timed_calls(torch, call, args.steps, max(1, args.warmup))
    # forward sections (read + write psi), H psi (read psi, write lambda), energy
    # (read psi), reverse sections (read + write psi and lambda)
    call_bytes = batch * (6.0 * S + 3.0) * (1 << n) * es
    ms = wall * 1e3 / args.steps
    log("adjoint: %.3f ms per call, E[0] = %.6f" % (ev_ms / args.steps, energy[0].item()))
    rec = {
        "metric": "adjoint gradients per second (20-qubit ansatz, 1600 parameters)",
        "value": round(batch * args.steps / wall, 2), "unit": "gradients/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if dt == B.QSV_C128 else "f32", "data": "synthetic",
        "config": {"workload": "hardware-efficient ansatz 20q x 40 layers (RY.RZ + CX ring), "
                               "batch %d, H = sum Z_i Z_i+1, %s, seed %d" % (batch, args.dtype, args.seed),
                   "sections": S, "chunk_bits": plan.stats()["chunk_bits"],
                   "register_bits": plan.stats()["register_bits"], "plan_s": round(t_plan, 3)},
        "roofline": {"bound": "hbm", "kernel": "qsv_adjoint_grad (forward + reverse sections)",
                     "achieved": round(call_bytes / (ev_ms / args.steps * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(call_bytes / (ev_ms / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "note": "algorithmic bytes per call = batch x (6 S + 3) x 2^n x es"},
        "autotune": tune_rec,
    }
    if not args.skip_cpu:
        import oracle
        ns, ls = 14, 40
        tm = W.hardware_efficient_ansatz(ns, ls)
        th = W.ansatz_parameters(ns, ls, 1, args.seed)[0]
        ts = [(1.0, (1 << i) | (1 << ((i + 1) % ns))) for i in range(ns)]
        t0 = time.perf_counter()
        reps = 0
        with one_thread():
            while reps == 0 or time.perf_counter() - t0 < 10.0:
                oracle.adjoint_gradient(ns, tm, th, ts)
                reps += 1
        dt_cpu = (time.perf_counter() - t0) / reps
        t_one = dt_cpu * float(1 << (n - ns))
        rec["cpu_baseline"] = {"value": round(1.0 / t_one, 5), "unit": "gradients/s",
                               "cores": 1, "kind": "oracle", "host_cores": len(os.sched_getaffinity(0)),
                               "sample": "oracle adjoint gradient of a 14-qubit 40-layer ansatz, %d "
                                         "evaluation(s) in %.1f s, scaled x2^6 amplitudes "
                                         "(extrapolated %.1f s per 20-qubit gradient)"
                                         % (reps, dt_cpu * reps, t_one)}
    print(json.dumps(rec), flush=True)


def bench_host(args, torch, B, W):
    """Quantum Volume with the state in pinned host memory: every section streams the
    state through HBM slice buffers (qsv_apply_host).  One step = `--sections`
    sections; value = host<->device bytes (state read + written per section) / time."""
    n = args.n
    dt = B.QSV_C128 if args.dtype == "c128" else B.QSV_C64
    tdt = torch.complex128 if dt == B.QSV_C128 else torch.complex64
    es = 16 if dt == B.QSV_C128 else 8
    gates = W.quantum_volume(n, n, args.seed)
    t0 = time.perf_counter()
    plan = B.Plan(n, gates, dt, diag_free=0)
    t_plan = time.perf_counter() - t0
    S = plan.stats()["n_sections"]
    ctx = B.Context(dt)
    t0 = time.perf_counter()
    host = torch.zeros(1 << n, dtype=tdt, pin_memory=True)
    host[0] = 1.0
    log("pinned host state of %d GiB ready in %.1f s" % ((es << n) >> 30, time.perf_counter() - t0))
    budget = int(args.hbm_budget_gib * (1 << 30))
    K = min(args.sections, S)
    ctx.apply_host(plan, host, budget, 0, 1)            # warm-up: the first section
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_read(0, reset=True)
    t1 = time.perf_counter()
    s0 = 1
    for _ in range(args.steps):
        s1 = min(S, s0 + K)
        if s1 - s0 < K:
            s0, s1 = 1, 1 + K
        ctx.apply_host(plan, host, budget, s0, s1)
        s0 = s1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    kern_ms, launches = ctx.timing_read(0, reset=True)
    ctx.timing(False)
    moved = 2.0 * (es << n) * K * args.steps
    o = 1
    while 3 * (es << (n - o)) > budget:
        o += 1
    rec = {
        "metric": "host-resident blocked apply: host<->HBM GB/s (state in pinned host memory), "
                  "%dq %s" % (n, args.dtype),
        "value": round(moved / wall / 1e9, 2), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": round(wall * 1e3 / args.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if dt == B.QSV_C128 else "f32", "data": "synthetic",
        "config": {"workload": "quantum-volume %dq depth %d, %s, seed %d, state in pinned host "
                               "memory (%d GiB), %d sections per step"
                               % (n, n, args.dtype, args.seed, (es << n) >> 30, K),
                   "sections": S, "hbm_budget_gib": args.hbm_budget_gib, "slices_per_section": 1 << o,
                   "plan_s": round(t_plan, 3)},
        "per_direction_gbs": round(moved / 2 / wall / 1e9, 2),
        "kernel_ms_per_section": round(kern_ms / max(1, launches) * (1 << o), 1),
        "roofline": {"bound": "host-link", "achieved": round(moved / 2 / wall / 1e9, 2),
                     "peak": 64.0, "unit": "GB/s", "frac": round(moved / 2 / wall / 1e9 / 64.0, 4),
                     "traffic": None,
                     "note": "per-direction host<->device bytes / time against PCIe 5.0 x16 "
                             "(64 GB/s per direction)"},
    }
    print(json.dumps(rec), flush=True)


def bench_density(args, torch, B, W):
    """A noisy circuit on an n-qubit density matrix (default 16 qubits: rho holds 2^32
    amplitudes, 64 GiB in complex128) through its 2n-qubit blocked plan (gates as U and
    conj(U), channels as superoperator gates).  One step = one application of the whole
    noisy circuit; value = sections x one pass of rho / wall time."""
    n = args.n
    dt = B.QSV_C128 if args.dtype == "c128" else B.QSV_C64
    tdt = torch.complex128 if dt == B.QSV_C128 else torch.complex64
    es = 16 if dt == B.QSV_C128 else 8
    layers = 8
    gates = W.noisy_density_circuit(n, layers, args.seed, p_depol=0.01, gamma=0.02, p_phase=0.005)
    opts = dict(chunk_bits=args.chunk_bits, pinned_low_bits=args.pinned,
                fusion_max_qubits=args.fusion, register_bits=args.register_bits,
                section_kernel=args.section_kernel, planner=args.planner)
    t0 = time.perf_counter()
    plan = B.Plan.density(n, gates, dt, **opts)
    t_plan = time.perf_counter() - t0
    st = plan.stats()
    S = st["n_sections"]
    N2 = 2 * n
    pass_bytes = 2.0 * (1 << N2) * es
    ctx = B.Context(dt)
    rho = torch.empty(1 << N2, dtype=tdt, device="cuda")
    ctx.dm_init_basis(rho, n, 0)
    for _ in range(max(1, args.warmup)):
        ctx.apply(plan, rho)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_read(0, reset=True)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        ctx.apply(plan, rho)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    sec_ms, launches = ctx.timing_read(0, reset=True)
    ctx.timing(False)
    tr = ctx.dm_trace(rho, n).item()
    purity = ctx.norm(rho, N2).item()
    avg_launch_ms = sec_ms / max(1, launches)
    rec = {
        "metric": "density-matrix noisy circuit: blocked apply GB/s (%% HBM peak), %dq rho "
                  "(%d-qubit plan) %s" % (n, N2, args.dtype),
        "value": round(S * pass_bytes * args.steps / wall / 1e9, 2), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if dt == B.QSV_C128 else "f32",
        "data": "synthetic",
        "config": {"workload": "%d-qubit density matrix, %d layers of U3 + depolarize(0.01), CX + "
                               "amplitude damping(0.02), phase damping(0.005), seed %d"
                               % (n, layers, args.seed),
                   "ops": len(gates), "sections": S, "chunk_bits": st["chunk_bits"],
                   "register_bits": st["register_bits"], "plan_s": round(t_plan, 3)},
        "trace_error": abs(tr - 1.0), "purity": purity,
        "ops_per_s": round(len(gates) * args.steps / wall, 1),
        "roofline": roofline(st, dt, B, args.steps, pass_bytes,
                             pass_bytes / (avg_launch_ms * 1e-3) / 1e9, avg_launch_ms, sec_ms,
                             launches, None, opts.get("section_kernel") or 0),
    }
    if not args.skip_cpu:
        with one_thread():
            import oracle
            ns = 6
            small = W.noisy_density_circuit(ns, layers, args.seed, p_depol=0.01, gamma=0.02,
                                            p_phase=0.005)
            t2 = time.perf_counter()
            reps = 0
            while time.perf_counter() - t2 < 10.0 or reps == 0:
                oracle.density.evolve(ns, small)
                reps += 1
            per_op = (time.perf_counter() - t2) / (reps * len(small))
            # the oracle multiplies full 2^n x 2^n operators: cost grows as 8^n
            t_full = per_op * len(gates) * 8.0 ** (n - ns)
        rec["cpu_baseline"] = {
            "value": S * pass_bytes / t_full / 1e9, "unit": "GB/s", "cores": 1,
            "host_cores": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": "oracle.density.evolve of the %d-qubit version of the circuit, %d run(s) "
                      "in %.1f s; time per op scaled x8^%d (full-operator products) x%d ops "
                      "(extrapolated %.3g s per step)" % (ns, reps, per_op * reps * len(small),
                                                          n - ns, len(gates), t_full)}
    print(json.dumps(rec), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2102_02957_amd import binding as B
    from paper_2102_02957_amd import workloads as W

    if args.workload == "trajectories":
        return bench_trajectories(args, torch, B, W)
    if args.workload == "adjoint":
        return bench_adjoint(args, torch, B, W)
    if args.workload == "host":
        if args.n is None:
            args.n = 32
        return bench_host(args, torch, B, W)
    if args.workload == "density":
        if args.n is None:
            args.n = 16
        return bench_density(args, torch, B, W)
    if args.n is None:
        args.n = 33

    n = args.n
    dt = B.QSV_C128 if args.dtype == "c128" else B.QSV_C64
    tdt = torch.complex128 if dt == B.QSV_C128 else torch.complex64
    es = 16 if dt == B.QSV_C128 else 8
    gates = W.quantum_volume(n, n, args.seed)
    torch.cuda.init()
    ctx = B.Context(dt)
    A = torch.empty(1 << n, dtype=tdt, device="cuda")

    def tune():
        cands = B.state_candidates(dt, n)
        best, ms = ctx.autotune(n, gates, candidates=cands, reps=1, scratch=A,
                                max_sections=TUNE_SECTIONS, refine=TUNE_REFINE)
        return best, cands, ms

    chosen, tune_rec = autotune(args, torch, B, dt, n, "quantum-volume depth %d seed %d"
                                % (n, args.seed), tune)
    if tune_rec.get("mode") in ("live", "cache"):
        tune_rec["max_sections"] = TUNE_SECTIONS
        tune_rec["refined"] = TUNE_REFINE
    opts = chosen or dict(chunk_bits=args.chunk_bits, pinned_low_bits=args.pinned,
                          fusion_max_qubits=args.fusion, register_bits=args.register_bits,
                          io_phases=args.io_phases, section_kernel=args.section_kernel,
                          planner=args.planner)
    t0 = time.perf_counter()
    plan = B.Plan(n, gates, dt, **opts)
    t_plan = time.perf_counter() - t0
    st = plan.stats()
    S = st["n_sections"]
    pass_bytes = 2.0 * (1 << n) * es
    step_bytes = S * pass_bytes
    log("planned n=%d gates=%d sections=%d phases=%d ops=%d in %.3f s"
        % (n, len(gates), S, st["n_phases"], st["n_device_ops"], t_plan))

    ctx.init_basis(A, n, 0)
    ctx.apply(plan, A)
    torch.cuda.synchronize()
    log("blocked apply #1 done")

    parity = {}
    pergate_ms = None
    if not args.skip_pergate:
        free, _ = torch.cuda.mem_get_info()
        Bst = None
        if free > A.numel() * es + (4 << 30):
            Bst = torch.empty(1 << n, dtype=tdt, device="cuda")
            ctx.init_basis(Bst, n, 0)
        else:
            Bst = A
            log("not enough memory for a second state: per-gate path timed on the same buffer")
        torch.cuda.synchronize()
        ctx.timing(True)
        t1 = time.perf_counter()
        ctx.apply(plan, Bst, B.QSV_MODE_PER_GATE)
        torch.cuda.synchronize()
        pergate_ms = (time.perf_counter() - t1) * 1e3
        pg_kernel_ms, pg_launches = ctx.timing_read(1, reset=True)
        ctx.timing(False)
        log("per-gate apply: %.1f ms (%d launches)" % (pergate_ms, pg_launches))
        if Bst is not A:
            ov = ctx.overlap(A, Bst, n).cpu().numpy()
            fid = (ov[0] ** 2 + ov[1] ** 2) / (ov[2] * ov[3])
            parity = {"one_minus_F_blocked_vs_pergate": float(1.0 - fid),
                      "norm_error": float(abs(ov[2] - 1.0))}
            log("parity: 1-F = %.3e, |norm-1| = %.3e" % (1.0 - fid, abs(ov[2] - 1.0)))
            del Bst
            torch.cuda.empty_cache()

    for _ in range(max(0, args.warmup - 1)):
        ctx.apply(plan, A)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_read(0, reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        ctx.apply(plan, A)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    sec_ms, sec_launches = ctx.timing_read(0, reset=True)
    ctx.timing(False)
    log("timed %d steps: %.1f ms/step" % (args.steps, wall * 1e3 / args.steps))

    nrm = ctx.norm(A, n).item()
    ms_per_step = wall * 1e3 / args.steps
    value = step_bytes * args.steps / wall / 1e9
    avg_launch_ms = sec_ms / max(1, sec_launches)
    achieved = pass_bytes / (avg_launch_ms * 1e-3) / 1e9

    # practical roofline: a plain streaming copy of 16 GiB through the same library
    copy_gbs = None
    try:
        nc = 30 if dt == B.QSV_C128 else 31
        X = torch.empty(1 << nc, dtype=tdt, device="cuda")
        Y = torch.empty(1 << nc, dtype=tdt, device="cuda")
        ctx.copy(Y, X, nc)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(5):
            ctx.copy(Y, X, nc)
        torch.cuda.synchronize()
        copy_gbs = 5 * 2.0 * (1 << nc) * es / (time.perf_counter() - t2) / 1e9
        del X, Y
    except Exception as e:  # pragma: no cover
        log("copy calibration skipped: %s" % e)

    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        with open(PROFILE_TRAFFIC) as f:
            prof = json.load(f)
        if (prof.get("kernel_source_hash") == kernel_source_hash() and prof.get("n") == n
                and prof.get("options") == {k: opts.get(k) for k in sorted(prof.get("options", {}))}):
            traffic = prof.get("bytes_per_launch")

    rec = {
        "metric": "blocked gate-apply GB/s (%% HBM peak) vs per-gate path, %dq %s at 1-F<%g"
                  % (n, args.dtype, 1e-12 if dt == B.QSV_C128 else 1e-5),
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dt == B.QSV_C128 else "f32",
        "data": "synthetic",
        "config": {
            "workload": "quantum-volume %dq depth %d, %s, seed %d, in place (%d GiB state)"
                        % (n, n, args.dtype, args.seed, (1 << n) * es >> 30),
            "gates": len(gates),
            "sections": S,
            "chunk_bits": st["chunk_bits"],
            "register_bits": st["register_bits"],
            "pinned_low_bits": st["pinned_low_bits"],
            "fusion_max_qubits": st["fusion_max_qubits"],
            "section_kernel": SECTION_KERNELS.get(opts.get("section_kernel") or 0),
            "planner": {None: "default", 0: "default", 1: "greedy", 2: "beam", 3: "exact"}.get(opts.get("planner"), "default"),
            "phases": st["n_phases"],
            "plan_s": round(t_plan, 4),
        },
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "gates_per_s": round(len(gates) * args.steps / wall, 2),
        "pergate_ms": None if pergate_ms is None else round(pergate_ms, 1),
        "speedup_vs_pergate": None if pergate_ms is None else round(pergate_ms / ms_per_step, 3),
        "pergate_gbs_algorithmic": None if pergate_ms is None else round(
            len(gates) * pass_bytes / (pergate_ms * 1e-3) / 1e9, 1),
        "copy_kernel_gbs": None if copy_gbs is None else round(copy_gbs, 1),
        "final_norm": nrm,
        "parity": parity,
        "roofline": roofline(st, dt, B, args.steps, pass_bytes, achieved, avg_launch_ms,
                             sec_ms, sec_launches, traffic, opts.get("section_kernel") or 0),
        "autotune": tune_rec,
    }
    if not args.skip_cpu:
        rec["cpu_baseline"] = cpu_baseline(n, gates, step_bytes, args.seed)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
