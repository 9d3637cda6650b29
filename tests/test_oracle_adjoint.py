"""The oracle's adjoint gradient against parameter shift, finite differences
and a closed form (CPU)."""

import math

import numpy as np
import pytest

import oracle
from paper_2102_02957_amd import workloads


@pytest.mark.parametrize("n,layers", [(3, 2), (4, 3), (6, 2)])
def test_adjoint_vs_shift_and_fd(n, layers):
    gates = workloads.hardware_efficient_ansatz(n, layers)
    theta = workloads.ansatz_parameters(n, layers, 1, 17 + n)[0]
    terms = oracle.ring_zz_terms(n)
    e, g = oracle.adjoint_gradient(n, gates, theta, terms)
    assert abs(e - oracle.energy(n, gates, theta, terms)) < 1e-13
    ps = oracle.parameter_shift_gradient(n, gates, theta, terms)
    fd = oracle.finite_difference_gradient(n, gates, theta, terms, h=1e-6)
    for p in range(len(theta)):
        assert abs(g[p] - ps[p]) < 1e-12
        assert abs(g[p] - fd[p]) < 1e-8


def test_product_ansatz_closed_form():
    """One layer of RY then RZ without CX: RZ changes no probability, so
    E = sum_i cos(a_i) cos(a_{i+1}) with a_i the RY angle of qubit i."""
    n = 5
    gates = [g for g in workloads.hardware_efficient_ansatz(n, 1) if g.kind != "cx"]
    theta = workloads.ansatz_parameters(n, 1, 1, 3)[0]
    terms = oracle.ring_zz_terms(n)
    e, g = oracle.adjoint_gradient(n, gates, theta, terms)
    a = theta[0::2]
    want_e = sum(math.cos(a[i]) * math.cos(a[(i + 1) % n]) for i in range(n))
    assert abs(e - want_e) < 1e-13
    for q in range(n):
        want = -math.sin(a[q]) * (math.cos(a[(q - 1) % n]) + math.cos(a[(q + 1) % n]))
        assert abs(g[2 * q] - want) < 1e-13
        assert abs(g[2 * q + 1]) < 1e-13


def test_shared_parameter_adds():
    """A parameter driving two gates: the adjoint sums both contributions
    (checked by finite differences, since the plain shift rule needs one use)."""
    n = 3
    gates = [("ry", (0,), (0.0,), None, 0), ("cx", (0, 1), (), None, -1),
             ("rx", (1,), (0.0,), None, 0), ("rz", (2,), (0.0,), None, 1),
             ("ry", (2,), (0.0,), None, 1), ("cx", (2, 0), (), None, -1)]
    theta = np.array([0.3, -1.1])
    terms = oracle.ring_zz_terms(n)
    _, g = oracle.adjoint_gradient(n, gates, theta, terms)
    fd = oracle.finite_difference_gradient(n, gates, theta, terms)
    assert abs(g[0] - fd[0]) < 1e-8 and abs(g[1] - fd[1]) < 1e-8


def test_parameter_shift_tail_equals_full_shift():
    """The prefix-sharing shift rule gives the plain shift rule's entries, for
    parameters anywhere in the circuit (first, middle, last layer)."""
    n, layers = 5, 4
    gates = workloads.hardware_efficient_ansatz(n, layers)
    theta = workloads.ansatz_parameters(n, layers, 1, 9)[0]
    terms = oracle.ring_zz_terms(n)
    picks = [0, 7, 2 * n * (layers - 1) + 3, 2 * n * layers - 1]
    full = oracle.parameter_shift_gradient(n, gates, theta, terms, indices=picks)
    tail = oracle.parameter_shift_tail(n, gates, theta, terms, picks)
    _, g = oracle.adjoint_gradient(n, gates, theta, terms)
    for p in picks:
        assert abs(tail[p] - full[p]) < 1e-13
        assert abs(tail[p] - g[p]) < 1e-12
