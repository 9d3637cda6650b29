"""Pins of the oracle's gate matrices and index arithmetic (CPU).

Everything here is checked against something other than the oracle itself:
the paper's printed Eq. (2), its worked pairing example, textbook matrices
typed out literally, and algebraic identities.
"""

import math

import numpy as np
import pytest

import oracle
from oracle.gates import gate_matrix, gate_derivative
from tests.conftest import read_golden

SQ = 1.0 / math.sqrt(2.0)
TEXTBOOK = {
    "h": np.array([[SQ, SQ], [SQ, -SQ]]),
    "x": np.array([[0, 1], [1, 0]]),
    "y": np.array([[0, -1j], [1j, 0]]),
    "z": np.array([[1, 0], [0, -1]]),
    "s": np.array([[1, 0], [0, 1j]]),
    "t": np.array([[1, 0], [0, (1 + 1j) * SQ]]),
}


@pytest.mark.parametrize("name", sorted(TEXTBOOK))
def test_named_matches_textbook(name):
    u, k = gate_matrix(name)
    assert k == 1
    assert np.allclose(u, TEXTBOOK[name], atol=1e-15)


def test_u3_special_values():
    """Eq. (1) reduces to familiar gates at special angles."""
    h = oracle.u3_matrix(math.pi / 2, 0.0, math.pi)
    assert np.allclose(h, TEXTBOOK["h"], atol=1e-15)
    x = oracle.u3_matrix(math.pi, 0.0, math.pi)
    assert np.allclose(x, TEXTBOOK["x"], atol=1e-15)
    for th in (0.3, 1.7, -2.2):
        c, s = math.cos(th / 2), math.sin(th / 2)
        assert np.allclose(oracle.u3_matrix(th, 0.0, 0.0), [[c, -s], [s, c]], atol=1e-15)
        assert np.allclose(oracle.u3_matrix(th, -math.pi / 2, math.pi / 2),
                           [[c, -1j * s], [-1j * s, c]], atol=1e-15)
    for la in (0.4, 2.9):
        assert np.allclose(oracle.u3_matrix(0.0, 0.0, la), np.diag([1, np.exp(1j * la)]), atol=1e-15)


def test_u3_phi_lambda_not_transposed():
    """With phi != lambda the off-diagonal phases sit where Eq. (1) puts them:
    e^{i lambda} in row 0 (column 1), e^{i phi} in row 1 (column 0)."""
    th, ph, la = 1.1, 0.3, 2.0
    u = oracle.u3_matrix(th, ph, la)
    assert np.isclose(u[0, 1], -np.exp(1j * la) * math.sin(th / 2))
    assert np.isclose(u[1, 0], np.exp(1j * ph) * math.sin(th / 2))
    assert np.isclose(u[1, 1], np.exp(1j * (ph + la)) * math.cos(th / 2))
    assert np.isclose(u[0, 0], math.cos(th / 2)) and u[0, 0].imag == 0.0


@pytest.mark.parametrize("kind,params", [
    ("h", ()), ("x", ()), ("y", ()), ("z", ()), ("s", ()), ("sdg", ()), ("t", ()), ("tdg", ()),
    ("rx", (0.7,)), ("ry", (1.3,)), ("rz", (2.1,)), ("p", (0.4,)), ("u3", (0.5, 1.5, 2.5)),
    ("cx", ()), ("cz", ()), ("cp", (0.9,)), ("swap", ())])
def test_unitary(kind, params):
    u, k = gate_matrix(kind, params)
    assert u.shape == (1 << k, 1 << k)
    assert np.max(np.abs(u.conj().T @ u - np.eye(1 << k))) < 1e-14


def test_cnot_eq2_from_paper():
    """Eq. (2) as printed: control = the higher bit.  CX(control=1, target=0)
    on a 2-qubit register, applied column by column to basis states."""
    eq2 = np.array([[float(v) for v in r] for r in read_golden("eq2_cnot.txt")])
    cols = []
    for j in range(4):
        psi = oracle.basis_state(2, j)
        oracle.apply_gate(psi, 2, ("cx", (1, 0), (), None, -1))
        cols.append(psi)
    assert np.array_equal(np.array(cols).T.real, eq2)


def test_cnot_swaps_half():
    """Sec. II-A: CNOT(c, t) swaps a(x_c=1, x_t=0) with a(x_c=1, x_t=1) and
    leaves every other amplitude in place."""
    n, c, t = 5, 3, 1
    psi = np.arange(1 << n, dtype=np.complex128)
    out = oracle.apply_gate(psi.copy(), n, ("cx", (c, t), (), None, -1))
    for i in range(1 << n):
        if (i >> c) & 1:
            assert out[i] == psi[i ^ (1 << t)]
        else:
            assert out[i] == psi[i]


def test_fig_u3_pairs():
    """Fig. "u3_gate" / the u3 kernel listing: pairs (i0, i0 + 2^k) for n=4, k=2."""
    rows = read_golden("u3_pairs_n4_k2.txt")
    pairs = [(int(i0), int(i1)) for _, i0, i1 in rows]
    n, k = 4, 2
    # the listing's index arithmetic, re-derived: insert a zero bit at k
    for i, (i0, i1) in enumerate(pairs):
        low = i & ((1 << k) - 1)
        assert ((i - low) << 1) + low == i0 and i0 + (1 << k) == i1
    # the oracle's X on qubit 2 exchanges exactly these pairs
    psi = np.arange(16, dtype=np.complex128)
    out = oracle.apply_gate(psi.copy(), n, ("x", (k,), (), None, -1))
    for i0, i1 in pairs:
        assert out[i0] == psi[i1] and out[i1] == psi[i0]
    assert 0b0011 ^ (1 << 2) == 0b0111 and (0b0011, 0b0111) in pairs


def test_pairwise_matches_general_matrix_path():
    rng = np.random.default_rng(7)
    n = 6
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    u = oracle.u3_matrix(0.3, 1.2, 2.3)
    for k in range(n):
        a = oracle.apply_1q_pairwise(psi.copy(), n, k, u)
        b = oracle.apply_matrix(psi.copy(), n, (k,), u)
        assert np.max(np.abs(a - b)) < 1e-15


@pytest.mark.parametrize("kind", ["rx", "ry", "rz", "p"])
def test_derivative_matches_difference_quotient(kind):
    th, h = 0.77, 1e-6
    up, _ = gate_matrix(kind, (th + h,))
    um, _ = gate_matrix(kind, (th - h,))
    assert np.max(np.abs((up - um) / (2 * h) - gate_derivative(kind, (th,)))) < 1e-9


def test_paper_figures():
    fig = {r[0]: r[1] for r in read_golden("paper_figures.txt")}
    es = int(fig["bytes_per_amp_double"])
    assert es == np.dtype(np.complex128).itemsize
    assert (1 << 50) * es == int(fig["n50_bytes"])
    assert (1 << int(fig["max_qubits_16GB_gpu"])) * es <= 16e9 < (1 << 30) * es
    assert (1 << int(fig["max_qubits_512GB_host"])) * es <= 512 * 2**30
    assert len(oracle.zero_state(int(fig["qb_array_n"]))) == int(fig["qb_array_len"])
    assert int(fig["fig_u3_pair_a"], 0) ^ (1 << int(fig["fig_u3_k"])) == int(fig["fig_u3_pair_b"], 0)
