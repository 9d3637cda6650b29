"""Density-matrix evolution with noise channels (TEST INFRASTRUCTURE ONLY).

The plain definition, on a 2^n x 2^n matrix (no vectorisation trick): a gate U
maps rho to U rho U^dagger, a channel with Kraus operators K_m maps rho to
sum_m K_m rho K_m^dagger, where every operator is first embedded into the full
2^n-dimensional space entry by entry (``full_operator``).  This is the
noise-model simulation and density-matrix method that the paper's simulator
offers beside the state vector (Sec. III-A).

Channel kinds and their Kraus operators (textbook definitions):
  amp_damp(gamma)     K0 = [[1, 0], [0, sqrt(1-gamma)]], K1 = [[0, sqrt(gamma)], [0, 0]]
  phase_damp(lambda)  K0 = [[1, 0], [0, sqrt(1-lambda)]], K1 = [[0, 0], [0, sqrt(lambda)]]
  depolarize(p)       sqrt(1-p) I, sqrt(p/3) X, sqrt(p/3) Y, sqrt(p/3) Z
  kraus               matrix = stack of M operators (M, 2^k, 2^k), local index as for gates
"""

import math

import numpy as np

from .gates import gate_matrix

CHANNELS = ("amp_damp", "phase_damp", "depolarize", "kraus")


def kraus_operators(kind, params=(), matrix=None):
    """List of 2^k x 2^k Kraus matrices of a channel gate."""
    if kind == "amp_damp":
        g = float(params[0])
        return [np.array([[1, 0], [0, math.sqrt(1 - g)]], dtype=np.complex128),
                np.array([[0, math.sqrt(g)], [0, 0]], dtype=np.complex128)]
    if kind == "phase_damp":
        lam = float(params[0])
        return [np.array([[1, 0], [0, math.sqrt(1 - lam)]], dtype=np.complex128),
                np.array([[0, 0], [0, math.sqrt(lam)]], dtype=np.complex128)]
    if kind == "depolarize":
        p = float(params[0])
        a, b = math.sqrt(1 - p), math.sqrt(p / 3)
        return [a * np.eye(2, dtype=np.complex128),
                b * np.array([[0, 1], [1, 0]], dtype=np.complex128),
                b * np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
                b * np.array([[1, 0], [0, -1]], dtype=np.complex128)]
    if kind == "kraus":
        return [np.asarray(k, dtype=np.complex128) for k in matrix]
    raise ValueError("not a channel: %r" % (kind,))


def full_operator(n, qubits, u):
    """The 2^n x 2^n matrix of the k-qubit operator u on `qubits`:
    entry [y, x] = u[sub(y), sub(x)] when y and x agree on every other qubit,
    else 0 (sub(x) = sum_j bit(q_j of x) << j)."""
    N = 1 << n
    x = np.arange(N)
    mask = 0
    for q in qubits:
        mask |= 1 << q
    sub = np.zeros(N, dtype=np.int64)
    for j, q in enumerate(qubits):
        sub |= ((x >> q) & 1) << j
    rest = x & ~mask
    M = np.zeros((N, N), dtype=np.complex128)
    for r in range(1 << len(qubits)):
        y = rest.copy()
        for j, q in enumerate(qubits):
            if (r >> j) & 1:
                y |= 1 << q
        M[y, x] = u[r, sub]
    return M


def basis_density(n, b=0):
    rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    rho[b, b] = 1.0
    return rho


def evolve(n, gates, rho=None):
    """rho_out after every gate / channel of the list, in order (rho defaults to |0><0|)."""
    rho = basis_density(n) if rho is None else np.array(rho, dtype=np.complex128, copy=True)
    for g in gates:
        kind, qubits, params, matrix = g[0], tuple(g[1]), g[2], g[3]
        if kind in CHANNELS:
            out = np.zeros_like(rho)
            for K in kraus_operators(kind, params, matrix):
                F = full_operator(n, qubits, K)
                out += F @ rho @ F.conj().T
            rho = out
        else:
            u, _ = gate_matrix(kind, params, matrix)
            F = full_operator(n, qubits, u)
            rho = F @ rho @ F.conj().T
    return rho


def trace(rho):
    return float(np.trace(rho).real)


def zstring_expval_rho(rho, n, terms):
    """Tr(rho H) for H = sum_t coeff_t prod_{i in zmask_t} Z_i."""
    i = np.arange(1 << n)
    h = np.zeros(1 << n)
    for c, m in terms:
        par = np.zeros(1 << n, dtype=np.int64)
        x = i & int(m)
        while np.any(x):
            par ^= x & 1
            x = x >> 1
        h += float(c) * (1 - 2 * par)
    return float(np.sum(np.real(np.diag(rho)) * h))
