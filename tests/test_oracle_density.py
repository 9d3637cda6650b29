"""The density-matrix oracle against the state-vector oracle, closed forms of
the standard channels and the defining properties of quantum channels (CPU)."""

import math

import numpy as np
import pytest

import oracle
from oracle import density as D
from paper_2102_02957_amd import workloads as W


def test_noiseless_equals_pure_state():
    """Without channels rho = |psi><psi|, psi from the per-gate state-vector oracle
    (a different code path: pairwise updates, not embedded full operators)."""
    n = 5
    gates = W.random_circuit(n, 40, 3, max_unitary_qubits=3)
    psi = oracle.apply_circuit(n, gates)
    rho = D.evolve(n, gates)
    assert np.max(np.abs(rho - np.outer(psi, psi.conj()))) < 1e-13


def test_full_operator_brute_force():
    """Embedding pinned by the tensor product: a gate on (1, 3) of 4 qubits equals
    I (x) A (x) I (x) B ordering by qubit, for a product A (x) B."""
    rng = np.random.default_rng(0)
    A = W.haar_unitary(rng, 2)
    Bm = W.haar_unitary(rng, 2)
    u = np.kron(Bm, A)          # local bit 0 = qubit 1 (A), local bit 1 = qubit 3 (B)
    I2 = np.eye(2)
    want = np.kron(np.kron(np.kron(Bm, I2), A), I2)   # qubit 3 (x) qubit 2 (x) qubit 1 (x) qubit 0
    assert np.max(np.abs(D.full_operator(4, (1, 3), u) - want)) < 1e-15


@pytest.mark.parametrize("k", [1, 3, 7])
def test_amplitude_damping_closed_form(k):
    g = 0.2
    rho = D.evolve(1, [("x", (0,), (), None, -1)] + [("amp_damp", (0,), (g,), None, -1)] * k)
    assert abs(rho[1, 1].real - (1 - g) ** k) < 1e-15
    assert abs(rho[0, 0].real - (1 - (1 - g) ** k)) < 1e-15
    rho = D.evolve(1, [("h", (0,), (), None, -1)] + [("amp_damp", (0,), (g,), None, -1)] * k)
    assert abs(rho[0, 1] - 0.5 * (1 - g) ** (k / 2)) < 1e-15


@pytest.mark.parametrize("k", [1, 4])
def test_depolarizing_closed_form(k):
    """(1-p) rho + p/3 (X rho X + Y rho Y + Z rho Z) = (1 - 4p/3) rho + (2p/3) I."""
    p = 0.15
    rng = np.random.default_rng(k)
    u = W.haar_unitary(rng, 2)
    rho0 = D.evolve(1, [("unitary", (0,), (), u, -1)])
    rho = D.evolve(1, [("depolarize", (0,), (p,), None, -1)] * k, rho0)
    f = (1 - 4 * p / 3) ** k
    want = f * rho0 + (1 - f) * np.eye(2) / 2
    assert np.max(np.abs(rho - want)) < 1e-15
    zero = D.evolve(1, [("depolarize", (0,), (p,), None, -1)] * k)
    assert abs(D.zstring_expval_rho(zero, 1, [(1.0, 1)]) - f) < 1e-15


def test_phase_damping_closed_form():
    lam = 0.3
    rho = D.evolve(1, [("h", (0,), (), None, -1)] + [("phase_damp", (0,), (lam,), None, -1)] * 2)
    assert abs(rho[0, 1] - 0.5 * (1 - lam)) < 1e-15
    assert abs(rho[0, 0] - 0.5) < 1e-15 and abs(rho[1, 1] - 0.5) < 1e-15


def random_kraus(rng, k, m):
    """A random trace-preserving channel: blocks of a Haar isometry."""
    d = 1 << k
    V = W.haar_unitary(rng, d * m)[:, :d]
    return np.stack([V[i * d:(i + 1) * d, :] for i in range(m)])


def test_channels_trace_preserving_hermitian_positive():
    rng = np.random.default_rng(5)
    n = 4
    gates = W.random_circuit(n, 20, 1, max_unitary_qubits=2)
    gates += [("kraus", (2, 0), (), random_kraus(rng, 2, 3), -1),
              ("amp_damp", (1,), (0.4,), None, -1), ("depolarize", (3,), (0.2,), None, -1),
              ("kraus", (1,), (), random_kraus(rng, 1, 2), -1)]
    rho = D.evolve(n, gates)
    assert abs(D.trace(rho) - 1.0) < 1e-13
    assert np.max(np.abs(rho - rho.conj().T)) < 1e-14
    assert np.min(np.linalg.eigvalsh(rho)) > -1e-13
    # a single-operator 'kraus' channel is that unitary
    u = W.haar_unitary(rng, 4)
    a = D.evolve(n, gates + [("kraus", (3, 1), (), u[None], -1)])
    b = D.evolve(n, gates + [("unitary", (3, 1), (), u, -1)])
    assert np.max(np.abs(a - b)) < 1e-14


def test_zstring_expval_rho_matches_pure():
    n = 5
    gates = W.random_circuit(n, 30, 9, max_unitary_qubits=2)
    terms = oracle.ring_zz_terms(n) + [(0.5, 0b10010)]
    psi = oracle.apply_circuit(n, gates)
    assert abs(D.zstring_expval_rho(D.evolve(n, gates), n, terms)
               - oracle.zstring_expval(psi, n, terms)) < 1e-13
