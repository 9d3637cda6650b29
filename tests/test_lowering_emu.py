"""Lowering check on the CPU: a plan's device tables executed by a plain C++
emulator (tests/lowering_emu.cpp), compared with the oracle.

The emulator applies the tables the way the section kernels read them: gather
through the section's position -> physical map, the ops of each register phase
on data positions, the transposition between phases (and a check that the LDS
write and read layouts of every transposition agree and are a bijection), the
scatter, the chunk swaps of materialise mode.  A mistake in the planner's
lowering (a wrong phase map, op position, fused matrix or swizzle table) shows
up here without a GPU.  The oracle (per-gate products, Sec. II-A) is the
reference; the identity blocked == original is the claim of Sec. IV-A.
"""

import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2102_02957_amd import binding as B
from paper_2102_02957_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2102_02957_amd")


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if not os.path.exists(os.path.join(PKG, "libqsv.so")):
        pytest.fail("libqsv.so not built (python -m paper_2102_02957_amd.build)")
    exe = str(tmp_path_factory.mktemp("emu") / "lowering_emu")
    cmd = ["g++", "-O2", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "lowering_emu.cpp"), "-o", exe, "-L" + PKG, "-lqsv",
           "-Wl,-rpath," + PKG]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def run_emu(exe, n, gates, psi0, dt=B.QSV_C128, **opts):
    o = B.make_options(dt, **opts)
    lines = ["%d %d" % (n, dt),
             " ".join(str(v) for v in (o.chunk_bits, o.pinned_low_bits, o.fusion_max_qubits,
                                       o.swap_mode, o.diag_free, o.register_bits, o.io_phases,
                                       o.planner, o.section_kernel)),
             str(len(gates))]
    for g in gates:
        p = list(g.params) + [0.0] * (3 - len(g.params))
        row = [str(B.KINDS[g.kind]), str(len(g.qubits))] + [str(q) for q in g.qubits]
        row += ["%.17g" % v for v in p]
        if g.matrix is not None:
            m = np.asarray(g.matrix, dtype=np.complex128).ravel()
            row += ["1"] + ["%.17g %.17g" % (z.real, z.imag) for z in m]
        else:
            row += ["0"]
        lines.append(" ".join(row))
    lines += ["%.17g %.17g" % (z.real, z.imag) for z in psi0]
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True)
    if r.returncode != 0:
        raise AssertionError(r.stdout[-500:] + r.stderr[-500:])
    v = np.array(r.stdout.split(), dtype=np.float64).reshape(-1, 2)
    return v[:, 0] + 1j * v[:, 1]


def random_state(n, seed):
    rng = np.random.default_rng(3000 + seed)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return psi / np.linalg.norm(psi)


CASES = [
    # n, circuit, options
    (8, "random", dict(chunk_bits=6, register_bits=3, fusion_max_qubits=2)),
    (9, "random", dict(chunk_bits=7, register_bits=4, fusion_max_qubits=3, pinned_low_bits=2)),
    (10, "random", dict(chunk_bits=8, register_bits=2, fusion_max_qubits=0, diag_free=1)),
    (10, "random", dict(chunk_bits=8, register_bits=4, fusion_max_qubits=4, io_phases=1)),
    (11, "random", dict(chunk_bits=9, register_bits=5, fusion_max_qubits=2,
                        swap_mode=B.QSV_SWAP_MATERIALIZE)),
    (11, "random", dict(chunk_bits=9, register_bits=3, planner=B.QSV_PLANNER_GREEDY)),
    (11, "random", dict(chunk_bits=9, register_bits=4, planner=B.QSV_PLANNER_BEAM)),
    (9, "random", dict(chunk_bits=6, register_bits=3, section_kernel=B.QSV_KERNEL_LDS,
                       fusion_max_qubits=3)),
    (12, "random", dict(chunk_bits=9, section_kernel=B.QSV_KERNEL_MFMA, fusion_max_qubits=5,
                        pinned_low_bits=3)),
    (12, "qv", dict(chunk_bits=9, register_bits=4, section_kernel=B.QSV_KERNEL_PAIRED)),
    (12, "qv", dict(chunk_bits=10, register_bits=4, fusion_max_qubits=2, io_phases=1)),
    (12, "qft", dict(chunk_bits=8, register_bits=4, diag_free=1, fusion_max_qubits=2)),
    (10, "u3cx", dict(chunk_bits=8, register_bits=4, section_kernel=B.QSV_KERNEL_PAIRED,
                      fusion_max_qubits=2)),
]


def circuit(kind, n, seed):
    if kind == "random":
        return W.random_circuit(n, 8 * n, 900 + seed, max_unitary_qubits=3)
    if kind == "qv":
        return W.quantum_volume(n, n, 900 + seed)
    if kind == "qft":
        return W.qft(n)
    return W.u3_cx_layers(n, 6, 900 + seed)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_lowered_tables_match_oracle(emu, case):
    n, kind, opts = CASES[case]
    gates = circuit(kind, n, case)
    psi0 = random_state(n, case)
    got = run_emu(emu, n, gates, psi0, **opts)
    want = oracle.apply_circuit(n, gates, psi0)
    assert np.max(np.abs(got - want)) < 1e-10


def test_emulator_comparison_has_teeth(emu):
    """The comparison has teeth: the emulated plan matches its own circuit and
    not the same circuit with one more gate (the check must fail there)."""
    n = 9
    gates = W.random_circuit(n, 60, 77, max_unitary_qubits=2)
    psi0 = random_state(n, 77)
    got = run_emu(emu, n, gates, psi0, chunk_bits=7, register_bits=3)
    assert np.max(np.abs(got - oracle.apply_circuit(n, gates, psi0))) < 1e-10
    other = gates + [W.Gate("ry", (4,), (0.3,))]
    assert np.max(np.abs(got - oracle.apply_circuit(n, other, psi0))) > 1e-3
