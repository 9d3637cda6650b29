"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times (default options), on properties that hold
at any size or on outputs the oracle computes one by one:

* QFT of a basis state, 26 qubits: sampled amplitudes against the closed form;
* 30 layers of U3 + CX matchings, 26 qubits: blocked vs per-gate on the
  device (FP64 overlap), and the mirror circuit C C^-1 back to |0...0>;
* Quantum Volume, 33 qubits complex128 (the headline workload, 128 GiB per
  state): blocked vs per-gate on the device, 1 - F < 1e-12.
"""

import numpy as np
import pytest

import oracle
from paper_2102_02957_amd import binding as B
from paper_2102_02957_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def tdtype(torch, dt):
    return torch.complex128 if dt == B.QSV_C128 else torch.complex64


def fidelity_dev(ctx, a, b, n):
    ov = ctx.overlap(a, b, n).cpu().numpy()
    return (ov[0] ** 2 + ov[1] ** 2) / (ov[2] * ov[3]), ov[2], ov[3]


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_qft26_closed_form(torch, dt):
    n = 26
    x = W.random_basis_index(n, 0)
    ctx = B.Context(dt)
    plan = B.Plan(n, W.qft(n), dt)
    st = torch.empty(1 << n, dtype=tdtype(torch, dt), device="cuda")
    ctx.init_basis(st, n, x)
    ctx.apply(plan, st)
    ys = np.random.default_rng(1).integers(0, 1 << n, 8192)
    got = st[torch.from_numpy(ys).cuda()].cpu().numpy().astype(np.complex128)
    want = oracle.closed_forms.qft_basis_amplitudes(n, x, ys)
    tol = 1e-13 if dt == B.QSV_C128 else 2e-7
    assert np.max(np.abs(got - want)) < tol
    assert abs(ctx.norm(st, n).item() - 1.0) < (1e-12 if dt == B.QSV_C128 else 1e-5)


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_u3cx26_blocked_vs_pergate_and_mirror(torch, dt):
    n = 26
    gates = W.u3_cx_layers(n, 30, 0)
    ctx = B.Context(dt)
    plan = B.Plan(n, gates, dt)
    a = torch.empty(1 << n, dtype=tdtype(torch, dt), device="cuda")
    b = torch.empty_like(a)
    ctx.init_basis(a, n, 0)
    ctx.init_basis(b, n, 0)
    ctx.apply(plan, a, B.QSV_MODE_BLOCKED)
    ctx.apply(plan, b, B.QSV_MODE_PER_GATE)
    f, na, nb = fidelity_dev(ctx, a, b, n)
    tol = 1e-12 if dt == B.QSV_C128 else 1e-5
    assert 1.0 - f < tol
    assert abs(na - 1.0) < (1e-12 if dt == B.QSV_C128 else 1e-5)
    mplan = B.Plan(n, W.mirror(gates), dt)
    ctx.init_basis(a, n, 0)
    ctx.apply(mplan, a)
    amp0 = a[0:1].cpu().numpy().astype(np.complex128)[0]
    assert 1.0 - abs(amp0) ** 2 < (1e-11 if dt == B.QSV_C128 else 1e-4)


def test_qv33_headline_blocked_vs_pergate(torch):
    n = 33
    free, _ = torch.cuda.mem_get_info()
    if free < 2 * (16 << n) + (8 << 30):
        pytest.skip("needs two 128 GiB states")
    gates = W.quantum_volume(n, n, 0)
    ctx = B.Context(B.QSV_C128)
    plan = B.Plan(n, gates, B.QSV_C128)
    a = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    ctx.init_basis(a, n, 0)
    ctx.apply(plan, a)
    b = torch.empty_like(a)
    ctx.init_basis(b, n, 0)
    ctx.apply(plan, b, B.QSV_MODE_PER_GATE)
    f, na, nb = fidelity_dev(ctx, a, b, n)
    del a, b
    torch.cuda.empty_cache()
    assert 1.0 - f < 1e-12
    assert abs(na - 1.0) < 1e-12 and abs(nb - 1.0) < 1e-12


def test_qft34_c64_closed_form_64bit_indices(torch):
    """34 qubits complex64 (128 GiB): amplitude indices beyond 2^32, sampled
    against the closed form of the QFT of a basis state."""
    n = 34
    free, _ = torch.cuda.mem_get_info()
    if free < (8 << n) + (8 << 30):
        pytest.skip("needs a 128 GiB state")
    x = W.random_basis_index(n, 3)
    ctx = B.Context(B.QSV_C64)
    plan = B.Plan(n, W.qft(n), B.QSV_C64)
    st = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    ctx.init_basis(st, n, x)
    ctx.apply(plan, st)
    rng = np.random.default_rng(2)
    ys = np.concatenate([rng.integers(0, 1 << n, 4096), (1 << n) - 1 - rng.integers(0, 1 << 20, 64)])
    got = st[torch.from_numpy(ys).cuda()].cpu().numpy().astype(np.complex128)
    want = oracle.closed_forms.qft_basis_amplitudes(n, x, ys)
    nrm = ctx.norm(st, n).item()
    del st
    torch.cuda.empty_cache()
    assert np.max(np.abs(got - want)) < 2e-8
    assert abs(nrm - 1.0) < 1e-5
