"""The C ABI's contract on the GPU: host-side validation before any launch,
numeric errors, workspaces shared by calls on two streams, and graph capture
of a reserved context (replays checked against the eager result)."""

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


def test_binding_rejects_mismatched_buffers(torch):
    """The C ABI sees pointers only; the binding checks dtype and shapes before
    any launch (a complex64 buffer given to a complex128 context would be read
    and written past its end)."""
    n = 8
    ctx = B.Context(B.QSV_C128)
    plan = B.Plan(n, W.ghz(n), B.QSV_C128)
    st64 = torch.zeros(1 << n, dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        ctx.init_basis(st64, n, 0)
    with pytest.raises(ValueError):
        ctx.apply(plan, st64)
    with pytest.raises(ValueError):
        ctx.norm(st64, n)
    tmpl = W.hardware_efficient_ansatz(n, 2)
    pplan = B.Plan(n, tmpl, B.QSV_C128)
    P = pplan.stats()["n_params"]
    st = torch.zeros(2 << n, dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):   # wrong parameter count
        ctx.apply_params(pplan, st, torch.zeros(2, P + 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):   # wrong parameter dtype
        ctx.apply_params(pplan, st, torch.zeros(2, P, dtype=torch.float32, device="cuda"))
    lam = torch.empty_like(st)
    with pytest.raises(ValueError):   # caller-supplied gradient of the wrong shape
        ctx.adjoint_grad(pplan, oracle.ring_zz_terms(n), torch.zeros(2, P, dtype=torch.float64,
                         device="cuda"), st, lam, grad=torch.empty(2, P - 1, dtype=torch.float64,
                                                                   device="cuda"))
    torch.cuda.synchronize()


def test_abi_rejects_unaligned_state_and_bad_terms(torch):
    n = 8
    ctx = B.Context(B.QSV_C128)
    buf = torch.zeros((1 << n) + 16, dtype=torch.complex128, device="cuda")
    view = buf[1:1 + (1 << n)]      # 16-byte offset: not 256-byte aligned
    with pytest.raises(B.QsvError) as e:
        ctx.init_basis(view, n, 0)
    assert e.value.status == -1 and "aligned" in str(e.value)
    st = buf[:1 << n]
    ctx.init_basis(st, n, 0)
    with pytest.raises(B.QsvError) as e:
        ctx.expval(st, n, [(float("nan"), 3)])
    assert e.value.status == -5
    with pytest.raises(B.QsvError) as e:
        ctx.expval(st, n, [(1.0, 1 << n)])
    assert e.value.status == -1
    torch.cuda.synchronize()


def test_expval_many_terms_async(torch):
    """More terms than one upload launch carries; the host list is dropped right
    after the call (no synchronisation happens inside it)."""
    n = 12
    ctx = B.Context(B.QSV_C128)
    gates = W.u3_cx_layers(n, 4, 3)
    plan = B.Plan(n, gates, B.QSV_C128, chunk_bits=9)
    st = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    ctx.init_basis(st, n, 0)
    ctx.apply(plan, st)
    rng = np.random.default_rng(0)
    terms = [(float(rng.standard_normal()), int(rng.integers(0, 1 << n))) for _ in range(300)]
    outs = []
    for k in range(3):
        outs.append(ctx.expval(st, n, list(terms[k * 100:(k + 1) * 100] + terms[:k])))
    full = ctx.expval(st, n, terms)
    psi = oracle.apply_circuit(n, gates)
    want = oracle.zstring_expval(psi, n, terms)
    assert abs(full.item() - want) < 1e-11 * max(1.0, abs(want))
    for k in range(3):
        w = oracle.zstring_expval(psi, n, terms[k * 100:(k + 1) * 100] + terms[:k])
        assert abs(outs[k].item() - w) < 1e-11 * max(1.0, abs(w))


def test_two_streams_share_workspaces(torch):
    """Parameter tables and reduction partials are context workspaces: calls on
    two streams are ordered by events, so interleaved launches on both streams
    give each stream's own results."""
    n, layers, batch = 12, 3, 4
    tmpl = W.hardware_efficient_ansatz(n, layers)
    plan = B.Plan(n, tmpl, B.QSV_C64, chunk_bits=9, register_bits=4)
    ctx = B.Context(B.QSV_C64)
    th = [W.ansatz_parameters(n, layers, batch, s) for s in (1, 2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    sts = [torch.empty(batch << n, dtype=torch.complex64, device="cuda") for _ in range(2)]
    pars = [torch.from_numpy(t).cuda() for t in th]
    norms = [torch.empty(1, dtype=torch.float64, device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    for rep in range(3):
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                for b in range(batch):
                    ctx.init_basis(sts[k][b << n:(b + 1) << n], n, 0)
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                ctx.apply_params(plan, sts[k], pars[k])
                ctx.norm(sts[k][:1 << n], n, out=norms[k])
    torch.cuda.synchronize()
    terms = oracle.ring_zz_terms(n)
    for k in range(2):
        out = sts[k].cpu().numpy().astype(np.complex128).reshape(batch, -1)
        assert abs(norms[k].item() - 1.0) < 1e-5
        for b in range(batch):
            want = oracle.apply_circuit(n, oracle.bind_params(tmpl, th[k][b]))
            assert 1.0 - oracle.fidelity(out[b], want) < 1e-5
            assert oracle.max_abs_diff(out[b], want) <= 2e-5 * np.max(np.abs(want))


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_graph_capture_after_reserve(torch, dt):
    """qsv_reserve, then qsv_apply_circuit + qsv_expval captured into a graph;
    every replay (eager work and synchronisation in between) matches the eager
    result bit for bit."""
    n = 16
    gates = W.quantum_volume(n, 8, 2)
    plan = B.Plan(n, gates, dt, chunk_bits=10)
    ctx = B.Context(dt)
    tdt = torch.complex128 if dt == B.QSV_C128 else torch.complex64
    terms = oracle.ring_zz_terms(n)
    eager = torch.empty(1 << n, dtype=tdt, device="cuda")
    ctx.init_basis(eager, n, 0)
    ctx.apply(plan, eager)
    e_eager = ctx.expval(eager, n, terms).clone()
    torch.cuda.synchronize()
    ctx.reserve(plan, batch=1)
    st = torch.empty(1 << n, dtype=tdt, device="cuda")
    e_out = torch.empty(1, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            ctx.init_basis(st, n, 0, stream=s)
            ctx.apply(plan, st, stream=s)
            ctx.expval(st, n, terms, out=e_out, stream=s)
    torch.cuda.synchronize()
    want = oracle.apply_circuit(n, gates)
    for rep in range(4):
        st.fill_(3.0)
        e_out.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(st, eager), rep
        assert e_out.item() == e_eager.item(), rep
        ctx.norm(eager, n)          # eager work between replays
    got = st.cpu().numpy().astype(np.complex128)
    tol = 1e-12 if dt == B.QSV_C128 else 1e-5
    assert 1.0 - oracle.fidelity(got, want) < tol
