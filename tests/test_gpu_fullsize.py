"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times (default options), on properties that hold
at any size or on outputs the oracle computes one by one:

* QFT of a basis state, 26 qubits: sampled amplitudes against the closed form;
* 30 layers of U3 + CX matchings, 26 qubits: blocked vs per-gate on the
  device (FP64 overlap), and the mirror circuit C C^-1 back to |0...0>;
* Quantum Volume, 33 qubits complex128 (the headline workload, 128 GiB per
  state): blocked vs per-gate on the device, 1 - F < 1e-12, and its mirror
  circuit back to |0...0>;
* QFT of a basis state, 33 qubits complex128: sampled amplitudes (indices
  beyond 2^32 included) against the closed form;
* Quantum-Volume layers inside three scattered qubit groups, 33 qubits
  complex128 and 34 qubits complex64: the state is a product of the groups'
  states, so sampled amplitudes are compared one by one with products of
  amplitudes the oracle computes on the small groups;
* Quantum Volume, 34 qubits complex64 (128 GiB): blocked vs per-gate with the
  FP64 device overlap (1 - F < 1e-5), and its mirror back to |0...0>.
"""

import gc

import numpy as np
import pytest

import oracle
from paper_2102_02957_amd import binding as B
from paper_2102_02957_amd import workloads as W

import grouped

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def tdtype(torch, dt):
    return torch.complex128 if dt == B.QSV_C128 else torch.complex64


@pytest.fixture(autouse=True)
def release_memory(torch):
    """Each full-size test holds up to 256 GiB: hand it back to the device
    before the next one."""
    yield
    gc.collect()
    torch.cuda.empty_cache()


def need_bytes(torch, nbytes):
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes + (6 << 30):
        pytest.skip("needs %.0f GiB of device memory" % (nbytes / 2 ** 30))


def sample_indices(n, seed, count=4096):
    """Uniform indices plus indices in the top 2^20 (beyond 2^32 for n >= 33)."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.integers(0, 1 << n, count),
                           (1 << n) - 1 - rng.integers(0, 1 << 20, 256),
                           np.arange(16)]).astype(np.int64)


def gather(torch, st, ys):
    return st[torch.from_numpy(ys).cuda()].cpu().numpy().astype(np.complex128)


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


def test_qv33_c128_mirror_to_zero(torch):
    """C then C^-1 (every gate inverted, reverse order) through the blocked path
    at the headline size returns |0...0>."""
    n = 33
    need_bytes(torch, 16 << n)
    gates = W.quantum_volume(n, n, 0)
    ctx = B.Context(B.QSV_C128)
    plan = B.Plan(n, W.mirror(gates), B.QSV_C128)
    st = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    ctx.init_basis(st, n, 0)
    ctx.apply(plan, st)
    ys = sample_indices(n, 5)
    got = gather(torch, st, ys)
    nrm = ctx.norm(st, n).item()
    del st
    assert abs(1.0 - abs(got[ys == 0][0]) ** 2) < 1e-12
    assert np.max(np.abs(got[ys != 0])) < 1e-7
    assert abs(nrm - 1.0) < 1e-12


def test_qft33_c128_closed_form(torch):
    n = 33
    need_bytes(torch, 16 << n)
    x = W.random_basis_index(n, 4)
    ctx = B.Context(B.QSV_C128)
    plan = B.Plan(n, W.qft(n), B.QSV_C128)
    st = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    ctx.init_basis(st, n, x)
    ctx.apply(plan, st)
    ys = sample_indices(n, 6)
    got = gather(torch, st, ys)
    nrm = ctx.norm(st, n).item()
    del st
    want = oracle.closed_forms.qft_basis_amplitudes(n, x, ys)
    assert np.max(np.abs(got - want)) < 1e-9 * np.max(np.abs(want))
    assert abs(nrm - 1.0) < 1e-12


@pytest.mark.parametrize("n,dt,sizes", [(33, B.QSV_C128, [11, 11, 11]),
                                        (34, B.QSV_C64, [12, 11, 11])])
def test_grouped_qv_fullsize_vs_oracle(torch, n, dt, sizes):
    """Quantum-Volume layers (depth n) inside three scattered qubit groups, in
    the benchmark's launch configuration (default options): sampled amplitudes
    against products of the oracle's group states, element by element."""
    es = 16 if dt == B.QSV_C128 else 8
    need_bytes(torch, es << n)
    gates, groups = W.grouped_quantum_volume(n, sizes, n, 1)
    ctx = B.Context(dt)
    plan = B.Plan(n, gates, dt)
    assert plan.stats()["n_sections"] > 10
    st = torch.empty(1 << n, dtype=tdtype(torch, dt), device="cuda")
    ctx.init_basis(st, n, 0)
    ctx.apply(plan, st)
    ys = sample_indices(n, 7)
    got = gather(torch, st, ys)
    nrm = ctx.norm(st, n).item()
    del st
    want = grouped.product_amplitudes(grouped.group_states(gates, groups), groups, ys)
    rel = 1e-10 if dt == B.QSV_C128 else 1e-4
    assert np.max(np.abs(got - want)) <= rel * np.max(np.abs(want))
    assert abs(nrm - 1.0) < (1e-12 if dt == B.QSV_C128 else 1e-5)


def test_qv34_c64_blocked_vs_pergate_and_mirror(torch):
    """The complex64 half of the headline workload: 34 qubits (128 GiB per
    state), blocked vs per-gate with the FP64 device overlap, then the mirror
    circuit back to |0...0>."""
    n = 34
    need_bytes(torch, 2 * (8 << n))
    gates = W.quantum_volume(n, n, 0)
    ctx = B.Context(B.QSV_C64)
    plan = B.Plan(n, gates, B.QSV_C64)
    a = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    ctx.init_basis(a, n, 0)
    ctx.apply(plan, a)
    ctx.init_basis(b, n, 0)
    ctx.apply(plan, b, B.QSV_MODE_PER_GATE)
    f, na, nb = fidelity_dev(ctx, a, b, n)
    del b
    gc.collect()
    torch.cuda.empty_cache()
    assert 1.0 - f < 1e-5
    assert abs(na - 1.0) < 1e-5 and abs(nb - 1.0) < 1e-5
    mplan = B.Plan(n, W.mirror(gates), B.QSV_C64)
    ctx.init_basis(a, n, 0)
    ctx.apply(mplan, a)
    ys = sample_indices(n, 8)
    got = gather(torch, a, ys)
    del a
    assert 1.0 - abs(got[ys == 0][0]) ** 2 < 1e-4
    assert np.max(np.abs(got[ys != 0])) < 1e-4


@pytest.mark.parametrize("n,dt,sizes", [(33, B.QSV_C128, [11, 11, 11]),
                                        (34, B.QSV_C64, [12, 11, 11])])
def test_grouped_qv_paired_beam_vs_oracle(torch, n, dt, sizes):
    """The same product-structured check in the paired-phase kernel with the
    beam-search planner (the options the benchmark's autotuner selects)."""
    es = 16 if dt == B.QSV_C128 else 8
    need_bytes(torch, es << n)
    gates, groups = W.grouped_quantum_volume(n, sizes, n, 2)
    ctx = B.Context(dt)
    plan = B.Plan(n, gates, dt, section_kernel=B.QSV_KERNEL_PAIRED, planner=B.QSV_PLANNER_BEAM)
    st = torch.empty(1 << n, dtype=tdtype(torch, dt), device="cuda")
    ctx.init_basis(st, n, 0)
    ctx.apply(plan, st)
    ys = sample_indices(n, 9)
    got = gather(torch, st, ys)
    nrm = ctx.norm(st, n).item()
    del st
    want = grouped.product_amplitudes(grouped.group_states(gates, groups), groups, ys)
    rel = 1e-10 if dt == B.QSV_C128 else 1e-4
    assert np.max(np.abs(got - want)) <= rel * np.max(np.abs(want))
    assert abs(nrm - 1.0) < (1e-12 if dt == B.QSV_C128 else 1e-5)


def test_qv33_paired_beam_mirror_and_vs_registers(torch):
    """QV33 complex128 in the paired kernel with the beam planner: its mirror
    returns |0...0>, and the circuit itself agrees with the register-phase kernel
    (FP64 device overlap)."""
    n = 33
    need_bytes(torch, 2 * (16 << n))
    gates = W.quantum_volume(n, n, 0)
    ctx = B.Context(B.QSV_C128)
    opts = dict(section_kernel=B.QSV_KERNEL_PAIRED, planner=B.QSV_PLANNER_BEAM)
    a = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    ctx.init_basis(a, n, 0)
    ctx.apply(B.Plan(n, gates, B.QSV_C128, **opts), a)
    ctx.init_basis(b, n, 0)
    ctx.apply(B.Plan(n, gates, B.QSV_C128), b)
    f, na, nb = fidelity_dev(ctx, a, b, n)
    del b
    gc.collect()
    torch.cuda.empty_cache()
    assert 1.0 - f < 1e-12 and abs(na - 1.0) < 1e-12
    ctx.init_basis(a, n, 0)
    ctx.apply(B.Plan(n, W.mirror(gates), B.QSV_C128, **opts), a)
    ys = sample_indices(n, 10)
    got = gather(torch, a, ys)
    del a
    assert abs(1.0 - abs(got[ys == 0][0]) ** 2) < 1e-12
    assert np.max(np.abs(got[ys != 0])) < 1e-7


@pytest.mark.parametrize("n,dt,sizes", [(33, B.QSV_C128, [11, 11, 11]),
                                        (34, B.QSV_C64, [12, 11, 11])])
def test_grouped_qv_mfma_f5_vs_oracle(torch, n, dt, sizes):
    """Fused blocks of up to 5 qubits applied as complex MFMA contractions at the
    full size of the headline configurations: sampled amplitudes, including indices
    beyond 2^32, against the product of small oracle runs."""
    es = 16 if dt == B.QSV_C128 else 8
    need_bytes(torch, es << n)
    gates, groups = W.grouped_quantum_volume(n, sizes, n, 4)
    ctx = B.Context(dt)
    plan = B.Plan(n, gates, dt, section_kernel=B.QSV_KERNEL_MFMA, fusion_max_qubits=5,
                  chunk_bits=12 if dt == B.QSV_C128 else 13, planner=B.QSV_PLANNER_BEAM)
    assert plan.stats()["fusion_max_qubits"] == 5
    st = torch.empty(1 << n, dtype=tdtype(torch, dt), device="cuda")
    ctx.init_basis(st, n, 0)
    ctx.apply(plan, st)
    ys = sample_indices(n, 11)
    got = gather(torch, st, ys)
    nrm = ctx.norm(st, n).item()
    del st
    want = grouped.product_amplitudes(grouped.group_states(gates, groups), groups, ys)
    rel = 1e-10 if dt == B.QSV_C128 else 1e-4
    assert np.max(np.abs(got - want)) <= rel * np.max(np.abs(want))
    assert abs(nrm - 1.0) < (1e-12 if dt == B.QSV_C128 else 1e-5)
