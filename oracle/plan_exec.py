"""Executor for an exported cache-blocked plan (TEST INFRASTRUCTURE ONLY).

It gives a transpiled op list its meaning (Sec. IV-A, the transpilation for
cache blocking, and Sec. IV-C, the chunk update loop) so that a plan can be
checked against the plain circuit:

  ('begin', local_mask)       begin_blocking: the next gates must act only on
                              the physical bits in local_mask (the chunk)
  ('end',)                    end_blocking
  ('swap', a, b)              chunk_swap of physical bits a and b: a noiseless
                              SWAP, i.e. amplitudes move
  ('gate', index, phys)       gate ``gates[index]`` applied on physical qubits
                              ``phys`` (same order as the gate's own tuple)

After the last op, logical qubit q sits at physical bit final_perm[q]; the
state is returned in logical order (Fig. "chunk_swap" case (b): reorder for
output).
"""

import numpy as np

from .gates import gate_matrix
from .statevector import apply_gate


def diagonal_qubit_positions(kind, params, matrix):
    """Positions j of the gate's qubit tuple in which its matrix is block
    diagonal (U[a, b] = 0 whenever bit j of a and b differ): a phase depends on
    that qubit (Sec. V-A: diagonal gates act on each amplitude on its own) or it
    is a control.  Such a qubit need not be in the chunk: its value is fixed
    per chunk when it is not local."""
    u, k = gate_matrix(kind, params, matrix)
    out = []
    for j in range(k):
        ok = True
        for a in range(1 << k):
            for b in range(1 << k):
                if ((a >> j) & 1) != ((b >> j) & 1) and u[a, b] != 0:
                    ok = False
        if ok:
            out.append(j)
    return out


def _unpermute(psi, n, final_perm):
    """out[x] = psi[y] with bit final_perm[q] of y equal to bit q of x."""
    if list(final_perm) == list(range(n)):
        return psi
    x = np.arange(1 << n, dtype=np.int64)
    y = np.zeros_like(x)
    for q in range(n):
        y |= ((x >> q) & 1) << int(final_perm[q])
    return psi[y]


def run_plan(n, gates, ops, final_perm, chunk_bits, diag_free=False, psi=None,
             check_local=True):
    """Execute ``ops`` on ``psi`` (default |0>), checking locality on the way.

    Raises AssertionError if a gate inside a section touches a non-local bit
    (with ``diag_free``, qubits in which the gate is block diagonal -- every
    qubit of a phase gate, the control of a CX -- are exempt), if a section's chunk does
    not hold exactly ``chunk_bits`` bits (fewer when n < chunk_bits), or if a
    gate is used a number of times other than once.
    """
    from .statevector import zero_state
    psi = zero_state(n) if psi is None else np.array(psi, dtype=np.complex128, copy=True)
    used = np.zeros(len(gates), dtype=np.int64)
    local = None
    for op in ops:
        tag = op[0]
        if tag == "begin":
            assert local is None, "nested begin_blocking"
            local = int(op[1])
            assert bin(local).count("1") == min(chunk_bits, n), "chunk must hold %d bits" % min(chunk_bits, n)
        elif tag == "end":
            assert local is not None, "end_blocking without begin"
            local = None
        elif tag == "swap":
            assert local is None, "chunk_swap inside a section"
            a, b = int(op[1]), int(op[2])
            apply_gate(psi, n, ("swap", (a, b), (), None, -1))
        elif tag == "gate":
            idx, phys = int(op[1]), tuple(int(q) for q in op[2])
            kind, qubits, params, matrix, pidx = gates[idx]
            assert len(phys) == len(qubits)
            if check_local:
                assert local is not None, "gate outside a section"
                exempt = diagonal_qubit_positions(kind, params, matrix) if diag_free else []
                for j, q in enumerate(phys):
                    if j not in exempt:
                        assert (local >> q) & 1, "gate %d touches non-local bit %d" % (idx, q)
            used[idx] += 1
            apply_gate(psi, n, (kind, phys, params, matrix, pidx))
        else:
            raise ValueError("unknown op %r" % (op,))
    assert local is None, "unterminated section"
    assert np.all(used == 1), "every gate must appear exactly once"
    return _unpermute(psi, n, final_perm)
