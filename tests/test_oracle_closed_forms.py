"""Oracle against closed forms and library routines (CPU)."""

import math

import numpy as np
import pytest

import oracle
from paper_2102_02957_amd import workloads


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_ghz(n):
    psi = oracle.apply_circuit(n, workloads.ghz(n))
    assert np.max(np.abs(psi - oracle.ghz_state(n))) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8])
def test_qft_equals_scaled_inverse_fft(n):
    """QFT(psi) = sqrt(N) * numpy.fft.ifft(psi) for any psi."""
    rng = np.random.default_rng(n)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    got = oracle.apply_circuit(n, workloads.qft(n), psi)
    want = math.sqrt(1 << n) * np.fft.ifft(psi)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("n", [3, 7, 10])
def test_qft_basis_closed_form(n):
    x = workloads.random_basis_index(n, n)
    got = oracle.apply_circuit(n, workloads.qft(n), oracle.basis_state(n, x))
    want = oracle.closed_forms.qft_basis_amplitudes(n, x, range(1 << n))
    assert np.max(np.abs(got - want)) < 1e-13


def test_qft_closed_form_large_n_phase_exact():
    """At 33 qubits the exact-integer phase reduction still holds the unit
    circle: |a| = 2^-16.5 and a(x, 0) is real."""
    n = 33
    a = oracle.qft_basis_amplitude(n, 123456789, 0)
    assert abs(a - 2 ** -16.5) < 1e-20
    b = oracle.qft_basis_amplitude(n, (1 << 32), 1)  # phase pi
    assert abs(b + 2 ** -16.5) < 1e-18


@pytest.mark.parametrize("builder", ["u3cx", "qv", "random"])
def test_mirror_is_identity(builder):
    n = 7
    if builder == "u3cx":
        gates = workloads.u3_cx_layers(n, 4, 1)
    elif builder == "qv":
        gates = workloads.quantum_volume(n, n, 2)
    else:
        gates = workloads.random_circuit(n, 60, 3)
    psi = oracle.apply_circuit(n, workloads.mirror(gates))
    assert 1.0 - oracle.fidelity(psi, oracle.zero_state(n)) < 1e-13


def test_haar_su4_properties():
    rng = np.random.default_rng(0)
    for _ in range(10):
        u = workloads.haar_su(rng, 4)
        assert np.max(np.abs(u.conj().T @ u - np.eye(4))) < 1e-13
        assert abs(np.linalg.det(u) - 1.0) < 1e-12


def test_expval_closed_forms():
    n = 6
    terms = oracle.ring_zz_terms(n)
    assert abs(oracle.zstring_expval(oracle.zero_state(n), n, terms) - n) < 1e-15
    assert abs(oracle.zstring_expval(oracle.ghz_state(n), n, terms) - n) < 1e-14
    rng = np.random.default_rng(1)
    th = rng.uniform(-math.pi, math.pi, n)
    gates = [("ry", (q,), (float(th[q]),), None, -1) for q in range(n)]
    psi = oracle.apply_circuit(n, gates)
    want = sum(math.cos(th[i]) * math.cos(th[(i + 1) % n]) for i in range(n))
    assert abs(oracle.zstring_expval(psi, n, terms) - want) < 1e-13


def test_overlap_and_fidelity():
    n = 5
    rng = np.random.default_rng(4)
    a = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    assert abs(oracle.overlap(a, a) - oracle.norm2(a)) < 1e-12
    assert abs(oracle.fidelity(a, 2.5j * a) - 1.0) < 1e-14
    b = oracle.basis_state(n, 3)
    assert abs(oracle.overlap(b, a) - a[3]) < 1e-15


def test_grouped_circuit_is_a_product_state():
    """The product assembly used at full size (tests/grouped.py) against the
    oracle's plain run of the whole circuit, every amplitude."""
    from paper_2102_02957_amd import workloads as W
    import grouped
    n = 9
    gates, groups = W.grouped_quantum_volume(n, [4, 3, 2], 5, 7)
    want = oracle.apply_circuit(n, gates)
    st = grouped.group_states(gates, groups)
    got = grouped.product_amplitudes(st, groups, np.arange(1 << n, dtype=np.uint64))
    assert np.max(np.abs(got - want)) < 1e-14
    # every qubit is used and every group is scattered
    assert sorted(q for g in groups for q in g) == list(range(n))
