"""Seeded synthetic circuits: the inputs of every test and benchmark.

This module only draws random numbers and writes gate lists; it computes no
gate matrix from its angles and applies nothing.  Both the GPU path and the
CPU oracle take its output as their input.

A gate is ``Gate(kind, qubits, params, matrix, pidx)``:
  kind    one of  h x y z s sdg t tdg rx ry rz p u3  cx cz cp swap  unitary
          or a noise channel (density-matrix plans only): amp_damp(gamma)
          phase_damp(lambda) depolarize(p) kraus(matrix = stack of operators)
  qubits  tuple of distinct qubit indices; qubit k is bit k of the amplitude
          index.  cx is (control, target); unitary is (q0, q1, ...) with q0 the
          least significant bit of the matrix's row/column index
  params  angles (u3: theta, phi, lambda; rx/ry/rz/p/cp: one angle)
  matrix  complex128 2^k x 2^k row-major for ``unitary``, else None
  pidx    index into a parameter vector for the angle (adjoint), else -1

Random numbers come from numpy.random.default_rng(seed) (PCG64) in the draw
order written in each function.

The workloads stand in for the paper's benchmark circuits (Sec. V-A: Quantum
Volume and the QFT), at the sizes of the configurations this library is
measured on.
"""

import math
from typing import NamedTuple, Optional, Tuple

import numpy as np


class Gate(NamedTuple):
    kind: str
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()
    matrix: Optional[np.ndarray] = None
    pidx: int = -1


TWO_PI = 2.0 * math.pi


def haar_unitary(rng, dim):
    """Haar-random U(dim): QR of a complex Ginibre matrix with the phases of
    R's diagonal moved into Q (Mezzadri's recipe)."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def haar_su(rng, dim):
    """Haar-random SU(dim): a Haar unitary divided by a root of its determinant."""
    u = haar_unitary(rng, dim)
    det = np.linalg.det(u)
    return u / det ** (1.0 / dim)


def u3_cx_layers(n, layers, seed):
    """Layers of U3 on every qubit, then CX on a random perfect matching.

    Draw order per layer: for q = 0..n-1 the three angles (theta, phi, lambda)
    ~ U[0, 2pi); then perm = rng.permutation(n) and CX(perm[2i], perm[2i+1])
    for i < n // 2 (odd n leaves perm[-1] idle).
    """
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            th, ph, la = rng.uniform(0.0, TWO_PI, size=3)
            gates.append(Gate("u3", (q,), (float(th), float(ph), float(la))))
        perm = rng.permutation(n)
        for i in range(n // 2):
            gates.append(Gate("cx", (int(perm[2 * i]), int(perm[2 * i + 1]))))
    return gates


def qft(n):
    """QFT: for j = n-1 .. 0: H(j), then CP(pi / 2^(j-k)) on (k, j) for
    k = j-1 .. 0; finally SWAP(i, n-1-i) for i < n // 2.  No randomness."""
    gates = []
    for j in range(n - 1, -1, -1):
        gates.append(Gate("h", (j,)))
        for k in range(j - 1, -1, -1):
            gates.append(Gate("cp", (k, j), (math.pi / float(1 << (j - k)),)))
    for i in range(n // 2):
        gates.append(Gate("swap", (i, n - 1 - i)))
    return gates


def random_basis_index(n, seed):
    """x ~ U{0 .. 2^n - 1}."""
    rng = np.random.default_rng(seed)
    return int(rng.integers(0, 1 << n, dtype=np.uint64))


def quantum_volume(n, depth, seed):
    """Quantum-Volume-style circuit: per layer perm = rng.permutation(n), then
    for i < n // 2 a Haar SU(4) on (perm[2i], perm[2i+1])."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(depth):
        perm = rng.permutation(n)
        for i in range(n // 2):
            u = haar_su(rng, 4)
            gates.append(Gate("unitary", (int(perm[2 * i]), int(perm[2 * i + 1])), (), u))
    return gates


def grouped_quantum_volume(n, sizes, depth, seed):
    """Quantum-Volume-style layers inside disjoint qubit groups.

    The n qubits are split by rng.permutation(n) into groups of the given sizes
    (group g = the next sizes[g] entries, so every group is scattered over the
    whole register).  Per layer, for each group in turn: perm = a permutation of
    the group's qubits, then a Haar SU(4) on consecutive pairs.  The final state
    is the tensor product of the groups' states, so any amplitude of a large
    instance is a product of amplitudes of small ones.
    Returns (gates, groups) with groups[g] = the group's qubits in order."""
    assert sum(sizes) == n
    rng = np.random.default_rng(seed)
    order = rng.permutation(n)
    groups, o = [], 0
    for k in sizes:
        groups.append([int(q) for q in order[o:o + k]])
        o += k
    gates = []
    for _ in range(depth):
        for grp in groups:
            perm = rng.permutation(len(grp))
            for i in range(len(grp) // 2):
                u = haar_su(rng, 4)
                gates.append(Gate("unitary", (grp[perm[2 * i]], grp[perm[2 * i + 1]]), (), u))
    return gates, groups


def noisy_density_circuit(n, layers, seed, p_depol=0.01, gamma=0.02, p_phase=0.0):
    """U3 + CX layers (as ``u3_cx_layers``) with noise channels for the
    density-matrix method: depolarize(p_depol) after every U3 on its qubit,
    amp_damp(gamma) on both qubits after every CX, and phase_damp(p_phase) on every
    qubit at the end of each layer when p_phase > 0."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            th, ph, la = rng.uniform(0.0, TWO_PI, 3)
            gates.append(Gate("u3", (q,), (float(th), float(ph), float(la))))
            gates.append(Gate("depolarize", (q,), (float(p_depol),)))
        perm = rng.permutation(n)
        for i in range(n // 2):
            a, b = int(perm[2 * i]), int(perm[2 * i + 1])
            gates.append(Gate("cx", (a, b)))
            gates.append(Gate("amp_damp", (a,), (float(gamma),)))
            gates.append(Gate("amp_damp", (b,), (float(gamma),)))
        if p_phase > 0:
            for q in range(n):
                gates.append(Gate("phase_damp", (q,), (float(p_phase),)))
    return gates


def ghz(n):
    gates = [Gate("h", (0,))]
    for q in range(n - 1):
        gates.append(Gate("cx", (q, q + 1)))
    return gates


_INVERSE_SELF = {"h", "x", "y", "z", "cx", "cz", "swap"}


def inverse_gate(g):
    """The inverse of one gate, as a gate (used to build mirror circuits)."""
    k = g.kind
    if k in _INVERSE_SELF:
        return g
    if k == "s":
        return g._replace(kind="sdg")
    if k == "sdg":
        return g._replace(kind="s")
    if k == "t":
        return g._replace(kind="tdg")
    if k == "tdg":
        return g._replace(kind="t")
    if k in ("rx", "ry", "rz", "p", "cp"):
        return g._replace(params=(-g.params[0],), pidx=-1)
    if k == "u3":
        th, ph, la = g.params
        return g._replace(params=(-th, -la, -ph))
    if k == "unitary":
        return g._replace(matrix=np.ascontiguousarray(np.conj(g.matrix).T))
    raise ValueError(k)


def mirror(gates):
    """C followed by C^-1: the identity circuit."""
    return list(gates) + [inverse_gate(g) for g in reversed(gates)]


_ONE_Q = ["h", "x", "y", "z", "s", "sdg", "t", "tdg", "rx", "ry", "rz", "p", "u3"]
_TWO_Q = ["cx", "cz", "cp", "swap"]


def random_circuit(n, ngates, seed, max_unitary_qubits=3, kinds=None):
    """A random mix of every gate kind on random qubits (test input).

    Draw order per gate: kind index, then qubits (rng.choice without
    replacement), then angles ~ U[0, 2pi), then (unitary) a Haar matrix.
    """
    rng = np.random.default_rng(seed)
    pool = list(kinds) if kinds is not None else _ONE_Q + _TWO_Q + ["unitary"]
    if n < 2:
        pool = [k for k in pool if k in _ONE_Q or k == "unitary"]
    gates = []
    for _ in range(ngates):
        kind = pool[int(rng.integers(0, len(pool)))]
        if kind in _ONE_Q:
            qs = (int(rng.integers(0, n)),)
        elif kind in _TWO_Q:
            qs = tuple(int(v) for v in rng.choice(n, size=2, replace=False))
        else:
            k = int(rng.integers(1, min(max_unitary_qubits, n) + 1))
            qs = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
        if kind == "u3":
            params = tuple(float(v) for v in rng.uniform(0.0, TWO_PI, size=3))
        elif kind in ("rx", "ry", "rz", "p", "cp"):
            params = (float(rng.uniform(0.0, TWO_PI)),)
        else:
            params = ()
        matrix = haar_unitary(rng, 1 << len(qs)) if kind == "unitary" else None
        gates.append(Gate(kind, qs, params, matrix))
    return gates


def noisy_trajectories(count, n_min, n_max, depth, p, seed):
    """Pauli-noise trajectories of random U3 + CX circuits.

    Returns a list of (n_b, gates).  Draw order: n_b ~ U{n_min..n_max} for all
    trajectories first; then per trajectory the circuit's own draws (same
    order as u3_cx_layers, from the same generator), and after every gate, for
    every qubit it touches in tuple order, u ~ U[0,1): if u < p, a Pauli X, Y
    or Z (by u < p/3, < 2p/3, else) is inserted on that qubit.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_min, n_max + 1, size=count)
    out = []
    for b in range(count):
        n = int(ns[b])
        gates = []
        for _ in range(depth):
            layer = []
            for q in range(n):
                th, ph, la = rng.uniform(0.0, TWO_PI, size=3)
                layer.append(Gate("u3", (q,), (float(th), float(ph), float(la))))
            perm = rng.permutation(n)
            for i in range(n // 2):
                layer.append(Gate("cx", (int(perm[2 * i]), int(perm[2 * i + 1]))))
            for g in layer:
                gates.append(g)
                for q in g.qubits:
                    u = float(rng.uniform())
                    if u < p:
                        kind = "x" if u < p / 3 else ("y" if u < 2 * p / 3 else "z")
                        gates.append(Gate(kind, (q,)))
        out.append((n, gates))
    return out


def hardware_efficient_ansatz(n, layers):
    """Parameterised template: per layer RY then RZ on every qubit, then a
    ring CX(i, (i+1) mod n) for i = 0..n-1.  Parameter index of the RY/RZ on
    qubit q in layer l: (l * n + q) * 2 + {0: RY, 1: RZ}."""
    gates = []
    for layer in range(layers):
        for q in range(n):
            base = (layer * n + q) * 2
            gates.append(Gate("ry", (q,), (0.0,), None, base))
            gates.append(Gate("rz", (q,), (0.0,), None, base + 1))
        if n > 1:
            for i in range(n):
                gates.append(Gate("cx", (i, (i + 1) % n)))
    return gates


def ansatz_parameters(n, layers, batch, seed):
    """theta ~ U[-pi, pi], shape (batch, 2 * n * layers)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-math.pi, math.pi, size=(batch, 2 * n * layers))
