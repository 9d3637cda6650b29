"""The oracle's plan executor on hand-written plans, and the two chunk_swap
cases of the paper (CPU)."""

import numpy as np
import pytest

import oracle
from paper_2102_02957_amd import workloads


def test_hand_plan_remap():
    """n=3, chunk of 2 bits.  Gates: H0, CX(0,2), H1.  Section 1 holds {0,1}
    and runs H0 and H1 (H1 commutes past CX(0,2)); section 2 holds {0,2} and
    runs CX(0,2).  No amplitude moves, so final_perm is the identity."""
    n = 3
    gates = [("h", (0,), (), None, -1), ("cx", (0, 2), (), None, -1), ("h", (1,), (), None, -1)]
    ops = [("begin", 0b011), ("gate", 0, (0,)), ("gate", 2, (1,)), ("end",),
           ("begin", 0b101), ("gate", 1, (0, 2)), ("end",)]
    got = oracle.run_plan(n, gates, ops, [0, 1, 2], 2)
    want = oracle.apply_circuit(n, gates)
    assert np.max(np.abs(got - want)) < 1e-15


def test_hand_plan_materialised():
    """Same circuit; the chunk is always physical {0,1}.  chunk_swap(1,2)
    brings logical qubit 2 to physical bit 1, so CX(0,2) runs on (0,1)
    physically, and the output is reordered by final_perm = [0, 2, 1]."""
    n = 3
    gates = [("h", (0,), (), None, -1), ("cx", (0, 2), (), None, -1), ("h", (1,), (), None, -1)]
    ops = [("begin", 0b011), ("gate", 0, (0,)), ("gate", 2, (1,)), ("end",),
           ("swap", 1, 2),
           ("begin", 0b011), ("gate", 1, (0, 1)), ("end",)]
    got = oracle.run_plan(n, gates, ops, [0, 2, 1], 2)
    want = oracle.apply_circuit(n, gates)
    assert np.max(np.abs(got - want)) < 1e-15


def test_rejects_nonlocal_gate():
    gates = [("h", (2,), (), None, -1)]
    with pytest.raises(AssertionError):
        oracle.run_plan(3, gates, [("begin", 0b011), ("gate", 0, (2,)), ("end",)], [0, 1, 2], 2)


def test_diag_free_admits_global_diagonal():
    gates = [("cp", (0, 2), (0.3,), None, -1)]
    ops = [("begin", 0b011), ("gate", 0, (0, 2)), ("end",)]
    with pytest.raises(AssertionError):
        oracle.run_plan(3, gates, ops, [0, 1, 2], 2)
    got = oracle.run_plan(3, gates, ops, [0, 1, 2], 2, diag_free=True,
                          psi=np.full(8, 8 ** -0.5, dtype=np.complex128))
    want = oracle.apply_circuit(3, gates, np.full(8, 8 ** -0.5))
    assert np.max(np.abs(got - want)) < 1e-15


def test_rejects_dropped_or_repeated_gate():
    gates = [("h", (0,), (), None, -1), ("h", (1,), (), None, -1)]
    with pytest.raises(AssertionError):
        oracle.run_plan(2, gates, [("begin", 0b11), ("gate", 0, (0,)), ("end",)], [0, 1], 2)
    with pytest.raises(AssertionError):
        oracle.run_plan(2, gates, [("begin", 0b11), ("gate", 0, (0,)), ("gate", 0, (0,)),
                                   ("gate", 1, (1,)), ("end",)], [0, 1], 2)


def _chunks(psi, nc):
    return psi.reshape(-1, 1 << nc)


def test_chunk_swap_case_a():
    """Fig. "chunk_swap" (a): sq0 < nc <= sq1.  Chunks pair up across bit sq1;
    in each pair, the half of one chunk with bit sq0 = 1 trades places with the
    half of the other chunk with bit sq0 = 0; nothing else moves."""
    n, nc, sq0, sq1 = 5, 3, 1, 4
    psi = np.arange(1 << n).astype(np.complex128)
    out = oracle.apply_gate(psi.copy(), n, ("swap", (sq0, sq1), (), None, -1))
    cin, cout = _chunks(psi, nc), _chunks(out, nc)
    hi = 1 << (sq1 - nc)
    moved = 0
    for ci in range(cin.shape[0]):
        partner = ci ^ hi
        for j in range(1 << nc):
            bit0 = (j >> sq0) & 1
            bit1 = (ci & hi) != 0
            if bit0 != bit1:
                assert cout[ci, j] == cin[partner, j ^ (1 << sq0)]
                moved += 1
            else:
                assert cout[ci, j] == cin[ci, j]
    assert moved == (1 << n) // 2


def test_chunk_swap_case_b():
    """Fig. "chunk_swap" (b): nc <= sq0 < sq1.  Of the four chunks that differ
    only in bits sq0, sq1, the two with (bit sq0, bit sq1) = (1,0) and (0,1)
    are exchanged whole."""
    n, nc, sq0, sq1 = 5, 2, 2, 4
    psi = np.arange(1 << n).astype(np.complex128)
    out = oracle.apply_gate(psi.copy(), n, ("swap", (sq0, sq1), (), None, -1))
    cin, cout = _chunks(psi, nc), _chunks(out, nc)
    b0, b1 = 1 << (sq0 - nc), 1 << (sq1 - nc)
    for ci in range(cin.shape[0]):
        x0, x1 = (ci & b0) != 0, (ci & b1) != 0
        if x0 != x1:
            assert np.array_equal(cout[ci], cin[ci ^ b0 ^ b1])
        else:
            assert np.array_equal(cout[ci], cin[ci])


def test_diagonal_qubit_positions():
    from oracle.plan_exec import diagonal_qubit_positions
    assert diagonal_qubit_positions("cx", (), None) == [0]          # control only
    assert diagonal_qubit_positions("cp", (0.3,), None) == [0, 1]
    assert diagonal_qubit_positions("h", (), None) == []
    assert diagonal_qubit_positions("rz", (0.2,), None) == [0]
    assert diagonal_qubit_positions("swap", (), None) == []
    # controlled-U built by hand: block diagonal in the control (bit 1)
    cu = np.eye(4, dtype=complex)
    cu[2:, 2:] = [[0, 1j], [1j, 0]]
    assert diagonal_qubit_positions("unitary", (), cu) == [1]


def test_cx_global_control_allowed_with_diag_free():
    gates = [("cx", (2, 0), (), None, -1)]
    ops = [("begin", 0b011), ("gate", 0, (2, 0)), ("end",)]
    with pytest.raises(AssertionError):
        oracle.run_plan(3, gates, ops, [0, 1, 2], 2)
    psi = np.arange(8).astype(np.complex128)
    got = oracle.run_plan(3, gates, ops, [0, 1, 2], 2, diag_free=True, psi=psi)
    assert np.array_equal(got, oracle.apply_circuit(3, gates, psi))
