"""Per-gate state-vector application (TEST INFRASTRUCTURE ONLY).

The definition the GPU path must reproduce:  psi_out = U_G ... U_1 |x0>,
applied one gate at a time, in circuit order, in complex128.  No blocking,
fusion or reordering happens here.
"""

import numpy as np

from .gates import gate_matrix


def zero_state(n):
    """|0...0>: amplitude 1 at index 0, zeros elsewhere (Sec. IV-C)."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def basis_state(n, x):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[int(x)] = 1.0
    return psi


def apply_1q_pairwise(psi, n, k, u):
    """A 2x2 matrix on qubit k (Sec. II-A, Fig. "u3_gate").

    Amplitudes pair up as (i0, i0 + 2^k) for every i0 whose bit k is 0; viewing
    the vector as shape (2^(n-k-1), 2, 2^k) the middle axis is exactly that bit.
    """
    v = psi.reshape(1 << (n - k - 1), 2, 1 << k)
    a0 = v[:, 0, :].copy()
    a1 = v[:, 1, :].copy()
    v[:, 0, :] = u[0, 0] * a0 + u[0, 1] * a1
    v[:, 1, :] = u[1, 0] * a0 + u[1, 1] * a1
    return psi


def apply_matrix(psi, n, qubits, u):
    """A 2^k x 2^k matrix on the qubit tuple ``qubits`` (local index rule of
    oracle.gates: qubits[0] is the least significant local bit).

    The vector is viewed as an n-axis tensor, C order, so tensor axis
    n-1-q holds bit q.  The gate's axes are brought to the front, most
    significant local bit first, contracted with U, and put back.
    """
    k = len(qubits)
    if len(set(qubits)) != k:
        raise ValueError("repeated qubit in %r" % (qubits,))
    t = psi.reshape((2,) * n)
    axes = [n - 1 - q for q in reversed(qubits)]
    front = np.moveaxis(t, axes, list(range(k)))
    shape = front.shape
    flat = front.reshape(1 << k, -1)
    out = (u @ flat).reshape(shape)
    back = np.moveaxis(out, list(range(k)), axes)
    psi[:] = back.reshape(-1)
    return psi


def _two_bit_view(psi, n, a, b):
    """View with axes (.., bit hi, .., bit lo, ..) for two distinct qubits."""
    lo, hi = min(a, b), max(a, b)
    v = psi.reshape(1 << (n - hi - 1), 2, 1 << (hi - lo - 1), 2, 1 << lo)
    return v, lo, hi


def apply_gate(psi, n, gate):
    """Apply one gate tuple ``(kind, qubits, params, matrix, pidx)`` in place."""
    kind, qubits, params, matrix = gate[0], tuple(int(q) for q in gate[1]), gate[2], gate[3]
    for q in qubits:
        if not 0 <= q < n:
            raise ValueError("qubit %d out of range for n=%d" % (q, n))
    if kind == "cx":
        # Eq. (2): swap amplitudes of (x_c=1, x_t=0) and (x_c=1, x_t=1).
        c, t = qubits
        v, lo, hi = _two_bit_view(psi, n, c, t)
        if c > t:
            a = v[:, 1, :, 0, :].copy()
            v[:, 1, :, 0, :] = v[:, 1, :, 1, :]
            v[:, 1, :, 1, :] = a
        else:
            a = v[:, 0, :, 1, :].copy()
            v[:, 0, :, 1, :] = v[:, 1, :, 1, :]
            v[:, 1, :, 1, :] = a
        return psi
    if kind == "swap":
        v, lo, hi = _two_bit_view(psi, n, qubits[0], qubits[1])
        a = v[:, 0, :, 1, :].copy()
        v[:, 0, :, 1, :] = v[:, 1, :, 0, :]
        v[:, 1, :, 0, :] = a
        return psi
    if kind in ("cp", "cz"):
        phase = -1.0 if kind == "cz" else np.exp(1j * float(params[0]))
        v, lo, hi = _two_bit_view(psi, n, qubits[0], qubits[1])
        v[:, 1, :, 1, :] *= phase
        return psi
    u, k = gate_matrix(kind, params, matrix)
    if k != len(qubits):
        raise ValueError("gate %s expects %d qubits, got %r" % (kind, k, qubits))
    if k == 1:
        return apply_1q_pairwise(psi, n, qubits[0], u)
    return apply_matrix(psi, n, qubits, u)


def bind_params(gates, theta):
    """Replace the angle of every gate with pidx >= 0 by theta[pidx]."""
    out = []
    for g in gates:
        kind, qubits, params, matrix, pidx = g
        if pidx is not None and pidx >= 0:
            params = (float(theta[pidx]),) + tuple(params[1:])
        out.append((kind, qubits, params, matrix, pidx))
    return out


def apply_circuit(n, gates, psi=None):
    """psi_out = U_G ... U_1 psi (psi defaults to |0>)."""
    psi = zero_state(n) if psi is None else np.array(psi, dtype=np.complex128, copy=True)
    for g in gates:
        apply_gate(psi, n, g)
    return psi
