"""Host-resident states (GPU memory as the cache of a state in pinned host
memory): results against the oracle and bit for bit against the same plan run
on a device-resident state."""

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


@pytest.mark.parametrize("n,dt,sizes,cut", [(24, B.QSV_C128, [8, 8, 8], 3),
                                            (26, B.QSV_C64, [9, 9, 8], 4)])
def test_host_resident_vs_oracle_and_device(torch, n, dt, sizes, cut):
    es = 16 if dt == B.QSV_C128 else 8
    gates, groups = W.grouped_quantum_volume(n, sizes, 12, 4)
    ctx = B.Context(dt)
    plan = B.Plan(n, gates, dt, diag_free=0)
    S = plan.stats()["n_sections"]
    assert S >= 2
    host = torch.zeros(1 << n, dtype=tdtype(torch, dt), pin_memory=True)
    host[0] = 1.0
    budget = 3 * (es << (n - cut))          # three slice buffers of 2^(n-cut) amplitudes
    k = S // 2
    ctx.apply_host(plan, host, budget, 0, k)      # two calls: sections [0, k) and [k, S)
    ctx.apply_host(plan, host, budget, k, S)
    torch.cuda.synchronize()
    dev = torch.empty(1 << n, dtype=tdtype(torch, dt), device="cuda")
    ctx.init_basis(dev, n, 0)
    ctx.apply(plan, dev)
    torch.cuda.synchronize()
    assert torch.equal(host, dev.cpu())           # same kernels, same chunks: bit for bit
    rng = np.random.default_rng(1)
    ys = np.concatenate([rng.integers(0, 1 << n, 4096), np.arange(8)]).astype(np.int64)
    got = host.numpy()[ys].astype(np.complex128)
    want = grouped.product_amplitudes(grouped.group_states(gates, groups), groups, ys)
    rel = 1e-10 if dt == B.QSV_C128 else 1e-4
    assert np.max(np.abs(got - want)) <= rel * np.max(np.abs(want))
    nrm = float(np.sum(np.abs(host.numpy().astype(np.complex128)) ** 2))
    assert abs(nrm - 1.0) < (1e-12 if dt == B.QSV_C128 else 1e-5)


def test_host_refusals(torch):
    n = 16
    ctx = B.Context(B.QSV_C128)
    host = torch.zeros(1 << n, dtype=torch.complex128, pin_memory=True)
    qft = B.Plan(n, W.qft(n), B.QSV_C128, chunk_bits=10, diag_free=1)
    with pytest.raises(B.QsvError) as e:      # diagonal gates on non-local qubits
        ctx.apply_host(qft, host, 1 << 20)
    assert e.value.status == -4
    qv = B.Plan(n, W.quantum_volume(n, 4, 0), B.QSV_C128, chunk_bits=12, diag_free=0)
    with pytest.raises(B.QsvError) as e:      # 2^5 slices of 2^11 < one chunk of 2^12
        ctx.apply_host(qv, host, 3 * (16 << 11))
    assert e.value.status == -4
    with pytest.raises(ValueError):
        ctx.apply_host(qv, torch.zeros(1 << n, dtype=torch.complex128), 1 << 30)
