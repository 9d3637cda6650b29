"""Gate matrices for the oracle (TEST INFRASTRUCTURE ONLY; see package header).

Index convention (Sec. II-A, Fig. "u3_gate"): qubit k is bit k (value 2^k) of
the amplitude index, zero-based, least significant first.  For a gate acting on
the qubit tuple (q0, q1, ..., q_{k-1}) the gate-local row/column index is
sum_j bit(q_j) << j, i.e. q0 is the least significant local bit.

Named gates and the order of their qubit tuples:
  1 qubit:  h x y z s sdg t tdg  rx(t) ry(t) rz(t) p(l)  u3(t, phi, l)
  2 qubits: cx(control, target)  cz(a, b)  cp(a, b; phi)  swap(a, b)
  k qubits: unitary(q0..q_{k-1}; matrix 2^k x 2^k, row-major, local index as above)
"""

import math

import numpy as np

GATE_ARITY = {
    "h": 1, "x": 1, "y": 1, "z": 1, "s": 1, "sdg": 1, "t": 1, "tdg": 1,
    "rx": 1, "ry": 1, "rz": 1, "p": 1, "u3": 1,
    "cx": 2, "cz": 2, "cp": 2, "swap": 2,
}

_DIAGONAL = {"z", "s", "sdg", "t", "tdg", "rz", "p", "cz", "cp"}


def is_diagonal_kind(kind):
    """True for the named gates whose matrix is diagonal (QFT phases, Sec. V-A)."""
    return kind in _DIAGONAL


def u3_matrix(theta, phi, lam):
    """Eq. (1) of the paper, taken literally.

    The paper writes the second angle as psi; it is OpenQASM's phi.  Rows are
    the output basis state (0, 1), columns the input one.
    """
    c = math.cos(theta / 2.0)
    s = math.sin(theta / 2.0)
    return np.array(
        [[c, -np.exp(1j * lam) * s],
         [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]],
        dtype=np.complex128)


def _cnot_eq2():
    """Eq. (2): CNOT with the higher of the two bits as control.

    With the local-index rule above the tuple is (target, control): local index
    = x_target + 2 * x_control, so rows/columns 2 and 3 (control = 1) swap.
    """
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = m[1, 1] = 1.0
    m[2, 3] = m[3, 2] = 1.0
    return m


def gate_matrix(kind, params=(), matrix=None):
    """Return (U, k): the 2^k x 2^k matrix of a gate in its own qubit order.

    For ``cx`` the returned matrix is in the order (control, target), i.e. the
    control is local bit 0 and the target local bit 1 -- built by relabelling
    Eq. (2), whose order is (target, control).
    """
    p = tuple(float(v) for v in params)
    if kind == "unitary":
        u = np.asarray(matrix, dtype=np.complex128)
        k = int(round(math.log2(u.shape[0])))
        if u.shape != (1 << k, 1 << k):
            raise ValueError("unitary matrix must be 2^k x 2^k")
        return u, k
    if kind == "h":
        return np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0), 1
    if kind == "x":
        return np.array([[0, 1], [1, 0]], dtype=np.complex128), 1
    if kind == "y":
        return np.array([[0, -1j], [1j, 0]], dtype=np.complex128), 1
    if kind == "z":
        return np.array([[1, 0], [0, -1]], dtype=np.complex128), 1
    if kind == "s":
        return np.diag([1, 1j]).astype(np.complex128), 1
    if kind == "sdg":
        return np.diag([1, -1j]).astype(np.complex128), 1
    if kind == "t":
        return np.diag([1, np.exp(1j * math.pi / 4)]).astype(np.complex128), 1
    if kind == "tdg":
        return np.diag([1, np.exp(-1j * math.pi / 4)]).astype(np.complex128), 1
    if kind == "rx":
        c, s = math.cos(p[0] / 2), math.sin(p[0] / 2)
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128), 1
    if kind == "ry":
        c, s = math.cos(p[0] / 2), math.sin(p[0] / 2)
        return np.array([[c, -s], [s, c]], dtype=np.complex128), 1
    if kind == "rz":
        return np.diag([np.exp(-0.5j * p[0]), np.exp(0.5j * p[0])]).astype(np.complex128), 1
    if kind == "p":
        return np.diag([1, np.exp(1j * p[0])]).astype(np.complex128), 1
    if kind == "u3":
        return u3_matrix(p[0], p[1], p[2]), 1
    if kind == "cx":
        # Eq. (2) is in order (target, control); swap the two local bits.
        perm = [0, 2, 1, 3]
        m = _cnot_eq2()
        return m[np.ix_(perm, perm)], 2
    if kind == "cz":
        return np.diag([1, 1, 1, -1]).astype(np.complex128), 2
    if kind == "cp":
        return np.diag([1, 1, 1, np.exp(1j * p[0])]).astype(np.complex128), 2
    if kind == "swap":
        m = np.zeros((4, 4), dtype=np.complex128)
        m[0, 0] = m[3, 3] = 1.0
        m[1, 2] = m[2, 1] = 1.0
        return m, 2
    raise ValueError("unknown gate kind %r" % (kind,))


def gate_derivative(kind, params):
    """d U / d theta for the single-angle rotations (adjoint gradient)."""
    t = float(params[0])
    c, s = math.cos(t / 2), math.sin(t / 2)
    if kind == "ry":
        return 0.5 * np.array([[-s, -c], [c, -s]], dtype=np.complex128)
    if kind == "rx":
        return 0.5 * np.array([[-s, -1j * c], [-1j * c, -s]], dtype=np.complex128)
    if kind == "rz":
        return np.diag([-0.5j * np.exp(-0.5j * t), 0.5j * np.exp(0.5j * t)]).astype(np.complex128)
    if kind == "p":
        return np.diag([0, 1j * np.exp(1j * t)]).astype(np.complex128)
    raise ValueError("no derivative for gate kind %r" % (kind,))
