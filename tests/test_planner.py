"""Host planner through the C ABI (CPU only: planning needs no GPU).

The exported blocked plan (chunk_swaps, begin/end of sections, gates on
physical qubits) is executed by the oracle's plan executor, which checks that
every in-section gate is chunk-local and that every gate runs once; the
result must equal the plain circuit (Sec. IV-A: blocking only reorders
commuting gates and inserts noiseless swaps)."""

import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2102_02957_amd import binding as B
from paper_2102_02957_amd import workloads as W


def plan_matches_circuit(n, gates, dt=B.QSV_C128, **kw):
    p = B.Plan(n, gates, dt, **kw)
    st = p.stats()
    ops = p.export()
    rng = np.random.default_rng(n)
    psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi0 /= np.linalg.norm(psi0)
    got = oracle.run_plan(n, gates, ops, st["final_perm"], st["chunk_bits"],
                          diag_free=bool(st["diag_free"]), psi=psi0)
    want = oracle.apply_circuit(n, gates, psi0)
    assert np.max(np.abs(got - want)) < 1e-12
    return st, ops


CASES = [
    ("u3cx", lambda n, s: W.u3_cx_layers(n, 6, s)),
    ("qv", lambda n, s: W.quantum_volume(n, n, s)),
    ("qft", lambda n, s: W.qft(n)),
    ("random", lambda n, s: W.random_circuit(n, 80, s, max_unitary_qubits=3)),
    ("ghz", lambda n, s: W.ghz(n)),
]


@pytest.mark.parametrize("name,builder", CASES)
@pytest.mark.parametrize("n,c", [(6, 3), (9, 4), (11, 6), (12, 12)])
@pytest.mark.parametrize("mode", [B.QSV_SWAP_REMAP, B.QSV_SWAP_MATERIALIZE])
def test_plan_equals_circuit(name, builder, n, c, mode):
    gates = builder(n, 3)
    st, ops = plan_matches_circuit(n, gates, chunk_bits=c, swap_mode=mode,
                                   register_bits=min(4, c), pinned_low_bits=min(1, c - 3) if c > 3 else 0)
    assert st["n_sections"] >= 1
    if n <= c:
        assert st["n_sections"] == 1
    if mode == B.QSV_SWAP_REMAP:
        assert st["final_perm"] == list(range(n))


@pytest.mark.parametrize("diag_free", [0, 1])
def test_qft_diag_free_fewer_sections(diag_free):
    n = 14
    st, _ = plan_matches_circuit(n, W.qft(n), chunk_bits=6, diag_free=diag_free,
                                 pinned_low_bits=0)
    if diag_free:
        assert st["n_sections"] <= 6
    else:
        assert st["n_sections"] > 6


def test_diagonal_only_circuit_single_section():
    n = 10
    gates = [("cp", (a, b), (0.1 * a + 0.01 * b,), None, -1)
             for a in range(n) for b in range(a + 1, n)]
    st, _ = plan_matches_circuit(n, gates, chunk_bits=4, diag_free=1, pinned_low_bits=0)
    assert st["n_sections"] == 1


def test_global_only_gates():
    """Every gate on qubits outside the first chunk."""
    n = 10
    gates = [("h", (q,), (), None, -1) for q in range(6, 10)] + [("cx", (9, 7), (), None, -1)]
    plan_matches_circuit(n, gates, chunk_bits=4, pinned_low_bits=0)


def test_c_equals_n_minus_1():
    n = 9
    plan_matches_circuit(n, W.quantum_volume(n, n, 1), chunk_bits=n - 1, register_bits=3)


def test_pinned_low_bits_always_local():
    n, c, L = 12, 6, 3
    p = B.Plan(n, W.quantum_volume(n, n, 4), B.QSV_C128, chunk_bits=c, pinned_low_bits=L,
               register_bits=3)
    for op in p.export():
        if op[0] == "begin":
            assert op[1] & ((1 << L) - 1) == (1 << L) - 1


@pytest.mark.parametrize("f", [0, 2, 3, 4])
def test_fusion_counts(f):
    n = 10
    gates = W.u3_cx_layers(n, 4, 2)
    p = B.Plan(n, gates, B.QSV_C128, chunk_bits=n, fusion_max_qubits=f, register_bits=4)
    st = p.stats()
    if f >= 2:
        assert st["n_device_ops"] < len(gates)
    assert st["n_sections"] == 1


def test_deterministic():
    n = 20
    g = W.quantum_volume(n, n, 7)
    a = B.Plan(n, g, B.QSV_C128).export()
    b = B.Plan(n, g, B.QSV_C128).export()
    assert a == b


def test_progress_every_section_nonempty():
    n = 16
    for gates in (W.qft(n), W.quantum_volume(n, n, 3), W.u3_cx_layers(n, 5, 3)):
        ops = B.Plan(n, gates, B.QSV_C128, chunk_bits=5, register_bits=3, pinned_low_bits=1).export()
        count = 0
        for op in ops:
            if op[0] == "begin":
                count = 0
            elif op[0] == "gate":
                count += 1
            elif op[0] == "end":
                assert count > 0


def test_section_counts_benchmark_circuits():
    """Blocking at the benchmark sizes: far fewer HBM passes than gates."""
    qv = B.Plan(33, W.quantum_volume(33, 33, 0), B.QSV_C128).stats()
    assert qv["n_gates"] == 528 and qv["n_sections"] < 100
    qft = B.Plan(26, W.qft(26), B.QSV_C128).stats()
    assert qft["n_sections"] <= 8


@pytest.mark.parametrize("bad,msg", [
    ([("h", (5,), (), None, -1)], "out of range"),
    ([("cx", (1, 1), (), None, -1)], "repeated"),
    ([("unitary", (0, 1), (), None, -1)], "without matrix"),
    ([("ry", (0,), (0.0,), None, -2)], None),
    ([("h", (0,), (), None, 3)], "bound parameter"),
])
def test_invalid_gates_rejected(bad, msg):
    if msg is None:
        B.Plan(4, bad, B.QSV_C128)  # param -2 means unbound: accepted
        return
    with pytest.raises(B.QsvError) as e:
        B.Plan(4, bad, B.QSV_C128)
    assert e.value.status == -1 and msg in str(e.value)


def test_invalid_options_rejected():
    with pytest.raises(B.QsvError):
        B.Plan(20, W.ghz(20), B.QSV_C128, chunk_bits=15)
    with pytest.raises(B.QsvError):
        B.Plan(20, W.ghz(20), B.QSV_C128, swap_mode=7)
    with pytest.raises(B.QsvError):
        B.Plan(35, [], B.QSV_C128)
    with pytest.raises(B.QsvError):
        B.Plan(20, W.ghz(20), 3)
    with pytest.raises(B.QsvError) as e:
        B.Plan(20, W.ghz(20), B.QSV_C128, chunk_bits=13, register_bits=3)
    assert "threads per workgroup" in str(e.value)


def test_empty_circuit():
    st, ops = plan_matches_circuit(5, [], chunk_bits=3)
    assert st["n_sections"] == 1


def test_header_symbols_exported():
    """Every function declared in include/qsv.h is exported by libqsv.so."""
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    hdr = open(os.path.join(root, "include", "qsv.h")).read()
    declared = set(re.findall(r"\b(qsv_[a-z_]+)\s*\(", hdr))
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = declared - exported
    assert not missing, missing
    assert set(B.EXPORTED) <= exported
    L = B.lib()
    for name in declared:
        getattr(L, name)


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(B.QsvError) as e:
        B.Context(B.QSV_C128)
    assert e.value.status in (-3, -1)


def test_launch_grid_limits_rejected():
    """A section launch has 2^(n-c) workgroups of 2^(c-r) work-items; shapes past
    the grid limits are refused at plan time instead of truncating the grid."""
    with pytest.raises(B.QsvError) as e:
        B.Plan(34, W.ghz(34), B.QSV_C64, chunk_bits=3, register_bits=2)
    assert e.value.status == -4 and "grid" in str(e.value)
    with pytest.raises(B.QsvError) as e:
        B.Plan(34, W.ghz(34), B.QSV_C128, chunk_bits=3, register_bits=3)
    assert e.value.status == -4
    # the largest shapes used elsewhere stay accepted
    B.Plan(34, W.ghz(34), B.QSV_C64, chunk_bits=13, register_bits=5)
    B.Plan(34, W.ghz(34), B.QSV_C64, chunk_bits=4, register_bits=3)


@pytest.mark.parametrize("bad", [
    [("ry", (0,), (float("nan"),), None, -1)],
    [("u3", (1,), (0.1, float("inf"), 0.0), None, -1)],
    [("unitary", (0,), (), np.array([[1, 0], [0, np.nan]], dtype=complex), -1)],
])
def test_non_finite_gates_numeric_error(bad):
    with pytest.raises(B.QsvError) as e:
        B.Plan(4, bad, B.QSV_C128)
    assert e.value.status == -5


@pytest.mark.parametrize("req,r,want", [(5, 4, 4), (5, 5, 4), (3, 2, 2), (3, 4, 3), (0, 4, 0), (1, 4, 1)])
def test_stats_report_applied_fusion_width(req, r, want):
    n = 10
    p = B.Plan(n, W.u3_cx_layers(n, 4, 2), B.QSV_C64, chunk_bits=8, register_bits=r,
               fusion_max_qubits=req)
    assert p.stats()["fusion_max_qubits"] == want


def test_incremental_build_tracks_headers(tmp_path, monkeypatch):
    """The developer's incremental build recompiles a source when a header is newer."""
    from paper_2102_02957_amd import build as bld
    src = tmp_path / "a.hip"
    src.write_text("// x\n")
    obj = tmp_path / "a.hip.o"
    assert bld._stale(str(obj), str(src))
    obj.write_text("")
    import os, time
    old = time.time() - 100
    os.utime(str(src), (old, old))
    monkeypatch.setattr(bld, "CSRC", str(tmp_path))
    monkeypatch.setattr(bld, "INCLUDE", str(tmp_path))
    assert not bld._stale(str(obj), str(src))
    h = tmp_path / "b.hpp"
    h.write_text("")
    os.utime(str(obj), (old + 10, old + 10))
    assert bld._stale(str(obj), str(src))


def test_density_plan_shape_and_validation():
    n = 5
    gates = W.noisy_density_circuit(n, 2, 0, 0.01, 0.02, 0.01)
    p = B.Plan.density(n, gates, B.QSV_C128, chunk_bits=8)
    st = p.stats()
    assert st["n"] == 2 * n and p.n == 2 * n
    # every circuit gate twice (row and column copies), every channel once
    nchan = sum(1 for g in gates if g[0] in ("amp_damp", "phase_damp", "depolarize"))
    assert st["n_gates"] == 2 * (len(gates) - nchan) + nchan
    with pytest.raises(B.QsvError) as e:      # channels need a density plan
        B.Plan(n, gates, B.QSV_C128)
    assert e.value.status == -4
    with pytest.raises(B.QsvError) as e:
        B.Plan.density(n, [("amp_damp", (0,), (1.5,), None, -1)], B.QSV_C128)
    assert e.value.status == -1
    with pytest.raises(B.QsvError) as e:
        B.Plan.density(18, [], B.QSV_C128)
    assert e.value.status == -1
    with pytest.raises(B.QsvError) as e:
        B.Plan.density(n, [("ry", (0,), (0.1,), None, 0)], B.QSV_C128)
    assert e.value.status == -4
    with pytest.raises(B.QsvError) as e:
        B.Plan.density(n, [("depolarize", (0,), (float("nan"),), None, -1)], B.QSV_C128)
    assert e.value.status == -5


def test_autotune_cache_roundtrip(tmp_path):
    """The JSON cache stores the chosen options and the candidate table per key,
    survives a reload, and a hit skips the tuner."""
    path = str(tmp_path / "sub" / "tune.json")
    c = B.AutotuneCache(path)
    key = B.AutotuneCache.key("gfx950", B.QSV_C64, 34, "quantum-volume")
    calls = []

    def run():
        calls.append(1)
        cands = [dict(chunk_bits=12), dict(chunk_bits=13)]
        return cands[1], cands, [2.0, float("inf")]

    e, hit = c.tune(key, run)
    assert not hit and e["chosen"] == {"chunk_bits": 13} and e["ms"] == [2.0, None]
    c2 = B.AutotuneCache(path)
    e2, hit2 = c2.tune(key, run)
    assert hit2 and e2 == e and len(calls) == 1
    assert key == "gfx950|c64|n=34|quantum-volume"


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_candidate_grids_are_plannable(dt):
    """Every candidate of the bench grids is accepted by the planner at its size."""
    n = 22
    g = W.quantum_volume(n, 4, 0)
    for kw in B.state_candidates(dt, n):
        B.Plan(n, g, dt, **kw)
    for kw in B.adjoint_candidates(dt, 20):
        B.Plan(20, W.hardware_efficient_ansatz(20, 2), dt, **kw)
    for kw in B.batch_candidates(dt):
        B.Plan(14, W.u3_cx_layers(14, 2, 0), dt, **kw)


def brute_min_sections(n, gates, c, pinned=0):
    """Minimum number of sections by breadth-first search over the sets of gates
    already run, written independently of the library: a section with chunk set C
    runs, in order, every remaining gate whose qubits lie in C and share no qubit
    with an earlier remaining gate that did not run."""
    from itertools import combinations
    G = len(gates)
    qs = [set(g[1]) for g in gates]
    chunks = [set(C) | set(range(pinned)) for C in combinations(range(pinned, n), c - pinned)]
    frontier, seen, depth = {frozenset()}, {frozenset()}, 0
    while frontier:
        depth += 1
        nxt = set()
        for done in frontier:
            for C in chunks:
                ran, blocked = set(done), set()
                for i in range(G):
                    if i in done:
                        continue
                    if not (qs[i] & blocked) and qs[i] <= C:
                        ran.add(i)
                    else:
                        blocked |= qs[i]
                ran = frozenset(ran)
                if len(ran) == G:
                    return depth
                if ran not in seen:
                    seen.add(ran)
                    nxt.add(ran)
        frontier = nxt
    return 0


@pytest.mark.parametrize("seed", range(6))
def test_exact_planner_is_optimal_and_correct(seed):
    """The exact planner's section count equals an independent brute force, is
    never above the heuristics, and its plan equals the circuit."""
    n, c = 6, 3
    gates = W.random_circuit(n, 14, 100 + seed, max_unitary_qubits=2)
    want = brute_min_sections(n, gates, c)
    counts = {}
    for name, pl in (("default", B.QSV_PLANNER_DEFAULT), ("greedy", B.QSV_PLANNER_GREEDY),
                     ("beam", B.QSV_PLANNER_BEAM), ("exact", B.QSV_PLANNER_EXACT)):
        st, _ = plan_matches_circuit(n, gates, chunk_bits=c, register_bits=2, pinned_low_bits=0,
                                     diag_free=0, planner=pl)
        counts[name] = st["n_sections"]
    assert counts["exact"] == want, (counts, want)
    assert counts["exact"] <= min(counts.values())
    assert counts["beam"] <= counts["default"]


@pytest.mark.parametrize("name,builder,n,c", [
    ("qv", lambda n: W.quantum_volume(n, n, 1), 16, 6),
    ("u3cx", lambda n: W.u3_cx_layers(n, 6, 2), 14, 5),
    ("qft", lambda n: W.qft(n), 14, 6),
])
def test_beam_planner_plans_equal_circuit(name, builder, n, c):
    gates = builder(n)
    st, _ = plan_matches_circuit(n, gates, chunk_bits=c, register_bits=3, pinned_low_bits=1,
                                 planner=B.QSV_PLANNER_BEAM)
    d = B.Plan(n, gates, B.QSV_C128, chunk_bits=c, register_bits=3, pinned_low_bits=1).stats()
    assert st["n_sections"] <= d["n_sections"]


def test_planner_option_validation():
    with pytest.raises(B.QsvError) as e:
        B.Plan(8, W.ghz(8), B.QSV_C128, planner=7)
    assert e.value.status == -1
    with pytest.raises(B.QsvError) as e:
        B.Plan(8, W.ghz(8), B.QSV_C128, planner=B.QSV_PLANNER_BEAM, swap_mode=B.QSV_SWAP_MATERIALIZE)
    assert e.value.status == -4
    with pytest.raises(B.QsvError) as e:
        B.Plan(12, W.quantum_volume(12, 12, 0), B.QSV_C128, planner=B.QSV_PLANNER_EXACT)
    assert e.value.status == -4      # 72 gates: above the exact planner's limit


def test_host_stream_schedule():
    """The cut bits of every section: o bits, none local in the section, the
    highest non-local ones; a budget needing more cut bits than a section leaves
    non-local is refused."""
    n, c, o = 20, 12, 3
    p = B.Plan(n, W.quantum_volume(n, n, 2), B.QSV_C128, chunk_bits=c, diag_free=0)
    masks = p.stream_bits(o)
    begins = [op[1] for op in p.export() if op[0] == "begin"]
    assert len(masks) == len(begins) == p.stats()["n_sections"]
    for m, local in zip(masks, begins):
        assert bin(m).count("1") == o and m & local == 0
        nonlocal_bits = [b for b in range(n) if not (local >> b) & 1]
        assert sorted(b for b in range(n) if (m >> b) & 1) == nonlocal_bits[-o:]
    with pytest.raises(B.QsvError) as e:
        p.stream_bits(n - c + 1)
    assert e.value.status == -4


def test_mfma_plan_validation_and_block_fusion():
    """Matrix-core plans: gates of up to 5 qubits, fusion up to 5, chunk_bits >= 9,
    no bound parameters; block fusion gathers commuting gates into fewer ops
    than fusing consecutive gates only."""
    n = 12
    rng = np.random.default_rng(0)
    g5 = [W.Gate("unitary", (0, 3, 5, 8, 11), (), W.haar_unitary(rng, 32))]
    p = B.Plan(n, g5, B.QSV_C128, chunk_bits=10, section_kernel=B.QSV_KERNEL_MFMA)
    assert p.stats()["register_bits"] == 10
    for bad in (dict(chunk_bits=8), dict(chunk_bits=10, gates=W.hardware_efficient_ansatz(n, 1))):
        gates = bad.pop("gates", g5)
        with pytest.raises(B.QsvError) as e:
            B.Plan(n, gates, B.QSV_C128, section_kernel=B.QSV_KERNEL_MFMA, **bad)
        assert e.value.status == -4
    qv = W.quantum_volume(20, 20, 0)
    st_l = B.Plan(20, qv, B.QSV_C64, chunk_bits=12, section_kernel=B.QSV_KERNEL_LDS,
                  fusion_max_qubits=5).stats()
    st_m = B.Plan(20, qv, B.QSV_C64, chunk_bits=12, section_kernel=B.QSV_KERNEL_MFMA,
                  fusion_max_qubits=5).stats()
    assert st_l["fusion_max_qubits"] == 4 and st_m["fusion_max_qubits"] == 5
    st_l4 = B.Plan(20, qv, B.QSV_C64, chunk_bits=12, section_kernel=B.QSV_KERNEL_LDS,
                   fusion_max_qubits=4).stats()
    st_m4 = B.Plan(20, qv, B.QSV_C64, chunk_bits=12, section_kernel=B.QSV_KERNEL_MFMA,
                   fusion_max_qubits=4).stats()
    assert st_m4["n_sections"] == st_l4["n_sections"]
    assert st_m4["n_device_ops"] < st_l4["n_device_ops"]
    assert st_m["n_device_ops"] < st_m4["n_device_ops"]


def test_lds_kernel_plan_validation():
    n = 10
    p = B.Plan(n, W.quantum_volume(n, n, 0), B.QSV_C128, chunk_bits=8,
               section_kernel=B.QSV_KERNEL_LDS)
    st = p.stats()
    assert st["register_bits"] == 8 and st["n_phases"] == st["n_sections"]
    with pytest.raises(B.QsvError) as e:
        B.Plan(n, W.hardware_efficient_ansatz(n, 1), B.QSV_C128, section_kernel=B.QSV_KERNEL_LDS)
    assert e.value.status == -4
    rng = np.random.default_rng(0)
    g5 = [W.Gate("unitary", (0, 1, 2, 3, 4), (), W.haar_unitary(rng, 32))]
    with pytest.raises(B.QsvError) as e:
        B.Plan(n, g5, B.QSV_C128, section_kernel=B.QSV_KERNEL_LDS)
    assert e.value.status == -4
    with pytest.raises(B.QsvError):
        B.Plan(n, W.ghz(n), B.QSV_C128, section_kernel=7)


def _min_two_wide_steps(pairs):
    """Fewest steps that run the 2-qubit gates `pairs` (in circuit order) two at a
    time, after fusing each chain of gates on one pair with nothing in between on
    either qubit: breadth-first search over the sets of chains already run (a chain
    may run once every chain it depends on has run in an earlier step)."""
    chains, last = [], {}
    deps = []
    for a, b in pairs:
        ta, tb = last.get(a), last.get(b)
        if ta is not None and ta == tb and chains[ta] == frozenset((a, b)):
            continue
        chains.append(frozenset((a, b)))
        deps.append({t for t in (ta, tb) if t is not None})
        last[a] = last[b] = len(chains) - 1
    full = (1 << len(chains)) - 1
    frontier, seen, steps = {0}, {0}, 0
    while full not in frontier:
        nxt = set()
        for done in frontier:
            ready = [t for t in range(len(chains)) if not (done >> t) & 1
                     and all((done >> d) & 1 for d in deps[t])]
            picks = [(x, y) for i, x in enumerate(ready) for y in ready[i + 1:]] or [(ready[0],)]
            for pick in picks:
                s = done
                for t in pick:
                    s |= 1 << t
                if s not in seen:
                    seen.add(s)
                    nxt.add(s)
        frontier = nxt
        steps += 1
    return steps


@pytest.mark.parametrize("seed", range(4))
def test_paired_phases_are_minimal(seed):
    """Paired plans run each section in the fewest phases of two fused gate chains
    (checked against a breadth-first search per section), and their exported plan
    equals the circuit."""
    n, c = 9, 6
    gates = W.quantum_volume(n, 6, 300 + seed)
    plan = B.Plan(n, gates, B.QSV_C128, chunk_bits=c, pinned_low_bits=0,
                  section_kernel=B.QSV_KERNEL_PAIRED)
    want, cur = 0, None
    for op in plan.export():
        if op[0] == "begin":
            cur = []
        elif op[0] == "gate":
            cur.append(tuple(op[2]))
        elif op[0] == "end":
            want += _min_two_wide_steps(cur)
    assert plan.stats()["n_phases"] == want
    st, _ = plan_matches_circuit(n, gates, chunk_bits=c, pinned_low_bits=0,
                                 section_kernel=B.QSV_KERNEL_PAIRED)
    assert st["n_phases"] == want
