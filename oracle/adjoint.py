"""Gradients of E(theta) = <psi(theta)|H|psi(theta)> (TEST INFRASTRUCTURE ONLY).

psi(theta) = U_G(theta) ... U_1(theta) |0>, H diagonal (Z-strings).  A gate
with ``pidx >= 0`` takes its angle from theta[pidx]; a parameter may drive
several gates, whose contributions add.

Three independent routes:
* ``adjoint_gradient`` -- forward pass, lambda = H psi, then one reverse sweep
  over the gates keeping two states: undo U_j on psi, form
  2 Re <lambda | dU_j/dtheta | psi_{j-1}>, undo U_j on lambda;
* ``parameter_shift_gradient`` -- [E(theta_j + pi/2) - E(theta_j - pi/2)] / 2,
  exact for gates exp(-i theta P / 2) with a Pauli P (rx, ry, rz);
* ``finite_difference_gradient`` -- central differences.

``parameter_shift_tail`` evaluates the same shift rule but applies the gates in
front of the first gate that a shifted parameter drives only once (that prefix
state does not depend on the shifted parameters); it makes a few entries at 20
qubits affordable when the parameters sit near the end of the circuit.
"""

import math

import numpy as np

from .gates import gate_matrix, gate_derivative
from .observables import zstring_expval, zz_diag_values
from .statevector import apply_circuit, bind_params, apply_1q_pairwise, apply_matrix


def energy(n, gates, theta, terms):
    psi = apply_circuit(n, bind_params(gates, theta))
    return zstring_expval(psi, n, terms)


def _apply_dense(psi, n, qubits, u):
    if len(qubits) == 1:
        return apply_1q_pairwise(psi, n, qubits[0], u)
    return apply_matrix(psi, n, tuple(qubits), u)


def adjoint_gradient(n, gates, theta, terms):
    """Returns (E, grad) with grad[p] = dE/dtheta_p."""
    bound = bind_params(gates, theta)
    psi = apply_circuit(n, bound)
    h = zz_diag_values(n, terms)
    e = float(np.sum((psi.real ** 2 + psi.imag ** 2) * h))
    lam = h * psi
    grad = np.zeros(len(theta), dtype=np.float64)
    for g in reversed(bound):
        kind, qubits, params, matrix, pidx = g
        u, _ = gate_matrix(kind, params, matrix)
        udag = u.conj().T
        _apply_dense(psi, n, tuple(qubits), udag)          # psi <- psi_{j-1}
        if pidx is not None and pidx >= 0:
            du = gate_derivative(kind, params)
            dpsi = _apply_dense(psi.copy(), n, tuple(qubits), du)
            grad[pidx] += 2.0 * float(np.vdot(lam, dpsi).real)
        _apply_dense(lam, n, tuple(qubits), udag)          # lambda <- U_j^dag lambda
    return e, grad


def parameter_shift_gradient(n, gates, theta, terms, indices=None):
    theta = np.asarray(theta, dtype=np.float64)
    idx = range(len(theta)) if indices is None else indices
    out = {}
    for p in idx:
        tp = theta.copy()
        tp[p] += math.pi / 2
        tm = theta.copy()
        tm[p] -= math.pi / 2
        out[p] = 0.5 * (energy(n, gates, tp, terms) - energy(n, gates, tm, terms))
    return out


def finite_difference_gradient(n, gates, theta, terms, h=1e-6, indices=None):
    theta = np.asarray(theta, dtype=np.float64)
    idx = range(len(theta)) if indices is None else indices
    out = {}
    for p in idx:
        tp = theta.copy()
        tp[p] += h
        tm = theta.copy()
        tm[p] -= h
        out[p] = (energy(n, gates, tp, terms) - energy(n, gates, tm, terms)) / (2 * h)
    return out


def parameter_shift_tail(n, gates, theta, terms, indices):
    """Parameter-shift entries {p: dE/dtheta_p} for p in `indices`, sharing the
    unshifted prefix state (see the module docstring)."""
    theta = np.asarray(theta, dtype=np.float64)
    idx = set(int(p) for p in indices)
    first = len(gates)
    for j, g in enumerate(gates):
        pidx = g[4] if len(g) > 4 else -1
        if pidx is not None and pidx >= 0 and pidx in idx:
            first = j
            break
    prefix = apply_circuit(n, bind_params(gates[:first], theta))
    out = {}
    for p in sorted(idx):
        es = []
        for sgn in (+1, -1):
            t = theta.copy()
            t[p] += sgn * math.pi / 2
            psi = apply_circuit(n, bind_params(gates[first:], t), prefix.copy())
            es.append(zstring_expval(psi, n, terms))
        out[p] = 0.5 * (es[0] - es[1])
    return out
