"""GPU parity of the density-matrix method: an n-qubit circuit with noise
channels, run as a 2n-qubit blocked plan on the device, against the oracle's
plain rho -> sum K rho K^dagger evolution, element by element; trace, purity
and Z-string expectations from the device reductions."""

import numpy as np
import pytest

import oracle
from oracle import density as D
from paper_2102_02957_amd import binding as B
from paper_2102_02957_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {B.QSV_C128: 1e-12, B.QSV_C64: 2e-6}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ctxs(torch):
    return {B.QSV_C128: B.Context(B.QSV_C128), B.QSV_C64: B.Context(B.QSV_C64)}


def run_density(torch, ctx, n, gates, dt, **opts):
    plan = B.Plan.density(n, gates, dt, **opts)
    tdt = torch.complex128 if dt == B.QSV_C128 else torch.complex64
    st = torch.empty(1 << (2 * n), dtype=tdt, device="cuda")
    ctx.dm_init_basis(st, n, 0)
    ctx.apply(plan, st)
    torch.cuda.synchronize()
    v = st.cpu().numpy().astype(np.complex128)
    # rho[i][j] at index i | (j << n): row-major reshape gives [j][i]
    return st, v.reshape(1 << n, 1 << n).T, plan


def random_kraus(rng, k, m):
    d = 1 << k
    V = W.haar_unitary(rng, d * m)[:, :d]
    return np.stack([V[i * d:(i + 1) * d, :] for i in range(m)])


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
@pytest.mark.parametrize("n,layers,c,f", [(3, 3, 4, 0), (5, 3, 8, 2), (7, 2, 9, 2), (8, 2, 10, 3)])
def test_noisy_circuit_vs_oracle(torch, ctxs, dt, n, layers, c, f):
    gates = W.noisy_density_circuit(n, layers, n, 0.02, 0.05, 0.03)
    st, rho, plan = run_density(torch, ctxs[dt], n, gates, dt, chunk_bits=c, fusion_max_qubits=f)
    want = D.evolve(n, gates)
    assert np.max(np.abs(rho - want)) < TOL[dt] * 10, np.max(np.abs(rho - want))
    ctx = ctxs[dt]
    tr = ctx.dm_trace(st, n).item()
    assert abs(tr - 1.0) < (1e-12 if dt == B.QSV_C128 else 1e-5)
    terms = oracle.ring_zz_terms(n) + [(0.25, 1)]
    e = ctx.dm_expval(st, n, terms).item()
    assert abs(e - D.zstring_expval_rho(want, n, terms)) < (1e-12 if dt == B.QSV_C128 else 1e-5)
    purity = ctx.norm(st, 2 * n).item()
    assert abs(purity - float(np.real(np.trace(want @ want)))) < (1e-12 if dt == B.QSV_C128 else 1e-5)
    assert plan.stats()["n_sections"] >= 1


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_general_kraus_and_all_gate_kinds(torch, ctxs, dt):
    """Every named gate kind (row copies as given, column copies conjugated) and
    general 1- and 2-qubit Kraus channels."""
    n = 6
    rng = np.random.default_rng(3)
    gates = W.random_circuit(n, 50, 4, max_unitary_qubits=2)
    gates += [W.Gate("kraus", (4, 1), (), random_kraus(rng, 2, 3)),
              W.Gate("kraus", (2,), (), random_kraus(rng, 1, 2)),
              W.Gate("y", (5,)), W.Gate("s", (0,)), W.Gate("tdg", (3,)),
              W.Gate("rx", (2,), (0.7,)), W.Gate("cp", (1, 5), (1.1,)),
              W.Gate("u3", (4,), (0.3, 1.2, -0.4)), W.Gate("phase_damp", (0,), (0.2,))]
    gates += W.random_circuit(n, 20, 5, max_unitary_qubits=3)
    _, rho, _ = run_density(torch, ctxs[dt], n, gates, dt, chunk_bits=9)
    want = D.evolve(n, gates)
    assert np.max(np.abs(rho - want)) < TOL[dt] * 10


def test_density_9q_default_options_vs_oracle(torch, ctxs):
    """9 density qubits (an 18-qubit state) with the default options, several
    sections: the diagonal and a row against the oracle."""
    n = 9
    gates = W.noisy_density_circuit(n, 4, 1, 0.01, 0.03)
    st, rho, plan = run_density(torch, ctxs[B.QSV_C128], n, gates, B.QSV_C128)
    want = D.evolve(n, gates)
    assert np.max(np.abs(np.diag(rho) - np.diag(want))) < 1e-12
    assert np.max(np.abs(rho[7] - want[7])) < 1e-12
    assert plan.stats()["n_sections"] > 1
