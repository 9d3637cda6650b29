"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (written here, from the precision targets of the path): complex128
1 - F < 1e-12, complex64 1 - F < 1e-5 (normalised fidelity, FP64 sums);
pure permutation circuits bit-exact.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2102_02957_amd import binding as B
from paper_2102_02957_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {B.QSV_C128: 1e-12, B.QSV_C64: 1e-5}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ctxs(torch):
    return {B.QSV_C128: B.Context(B.QSV_C128), B.QSV_C64: B.Context(B.QSV_C64)}


def tdtype(torch, dt):
    return torch.complex128 if dt == B.QSV_C128 else torch.complex64


def to_dev(torch, psi, dt):
    return torch.from_numpy(np.asarray(psi, dtype=np.complex128)).to(tdtype(torch, dt)).cuda().contiguous()


def random_state(n, seed):
    rng = np.random.default_rng(1000 + seed)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return psi / np.linalg.norm(psi)


def run_gpu(torch, ctxs, n, gates, dt, psi0=None, mode=B.QSV_MODE_BLOCKED, **opts):
    plan = B.Plan(n, gates, dt, **opts)
    ctx = ctxs[dt]
    if psi0 is None:
        st = torch.empty(1 << n, dtype=tdtype(torch, dt), device="cuda")
        ctx.init_basis(st, n, 0)
    else:
        st = to_dev(torch, psi0, dt)
    ctx.apply(plan, st, mode)
    torch.cuda.synchronize()
    return st.cpu().numpy().astype(np.complex128), plan


# element-wise bound on max|got - want|, relative to the largest expected
# amplitude: far above the rounding of the dtype over a few hundred gates, far
# below what a wrong phase or a wrong matrix entry in any one gate produces
MAXD = {B.QSV_C128: 1e-11, B.QSV_C64: 2e-5}


def assert_close(got, want, dt, what=""):
    f = oracle.fidelity(got, want)
    err = 1.0 - f
    d = oracle.max_abs_diff(got, want)
    scale = float(np.max(np.abs(want))) if len(want) else 1.0
    assert err < TOL[dt], "%s: 1-F = %.3e, max|d| = %.3e" % (what, err, d)
    assert d <= MAXD[dt] * scale, "%s: max|d| = %.3e (scale %.3e), 1-F = %.3e" % (what, d, scale, err)
    assert abs(oracle.norm2(got) - 1.0) < (1e-12 if dt == B.QSV_C128 else 1e-5)


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
@pytest.mark.parametrize("mode", [B.QSV_MODE_BLOCKED, B.QSV_MODE_PER_GATE])
def test_config_plain_12q(torch, ctxs, dt, mode):
    """12 qubits, 20 layers of U3 on every qubit + CX on a random matching."""
    n = 12
    gates = W.u3_cx_layers(n, 20, 0)
    got, _ = run_gpu(torch, ctxs, n, gates, dt, mode=mode)
    assert_close(got, oracle.apply_circuit(n, gates), dt, "c1")


RANDOM_CASES = [
    # n, chunk_bits, register_bits, pinned, fusion, seed
    (1, 0, 0, 0, 0, 0),
    (2, 0, 0, 0, 2, 1),
    (3, 2, 1, 0, 0, 2),
    (5, 3, 2, 0, 2, 3),
    (7, 4, 2, 1, 2, 4),
    (9, 6, 3, 2, 3, 5),
    (10, 8, 4, 3, 4, 6),
    (13, 12, 4, 3, 2, 7),
    (14, 9, 4, 2, 0, 8),
    (16, 12, 4, 3, 2, 9),
    (17, 11, 5, 4, 3, 10),
    (18, 13, 5, 4, 4, 11),
    (19, 13, 4, 3, 2, 12),   # 2^9 threads per workgroup
]


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
@pytest.mark.parametrize("n,c,r,L,f,seed", RANDOM_CASES)
def test_random_circuits(torch, ctxs, dt, n, c, r, L, f, seed):
    gates = W.random_circuit(n, 6 * n + 10, seed, max_unitary_qubits=min(3, n))
    psi0 = random_state(n, seed)
    opts = dict(fusion_max_qubits=f)
    if c:
        opts.update(chunk_bits=c, register_bits=r, pinned_low_bits=L)
    want = oracle.apply_circuit(n, gates, psi0)
    got, _ = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, **opts)
    assert_close(got, want, dt, "blocked")
    got2, _ = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, mode=B.QSV_MODE_PER_GATE, **opts)
    assert_close(got2, want, dt, "per-gate")


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
@pytest.mark.parametrize("k", [4, 5])
def test_wide_unitaries(torch, ctxs, dt, k):
    n = 12
    rng = np.random.default_rng(k)
    gates = []
    for _ in range(6):
        qs = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
        gates.append(W.Gate("unitary", qs, (), W.haar_unitary(rng, 1 << k)))
    psi0 = random_state(n, k)
    want = oracle.apply_circuit(n, gates, psi0)
    got, _ = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, chunk_bits=10, register_bits=k)
    assert_close(got, want, dt)
    got, _ = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, mode=B.QSV_MODE_PER_GATE)
    assert_close(got, want, dt)


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
@pytest.mark.parametrize("mode", [B.QSV_MODE_BLOCKED, B.QSV_MODE_PER_GATE])
@pytest.mark.parametrize("swap_mode", [B.QSV_SWAP_REMAP, B.QSV_SWAP_MATERIALIZE])
def test_permutation_circuits_bit_exact(torch, ctxs, dt, mode, swap_mode):
    """X, CX and SWAP only move amplitudes: the result is bit-identical."""
    n = 15
    gates = W.random_circuit(n, 120, 21, kinds=["x", "cx", "swap"])
    psi0 = random_state(n, 3)
    if dt == B.QSV_C64:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    want = oracle.apply_circuit(n, gates, psi0)
    got, _ = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, mode=mode, chunk_bits=8,
                     register_bits=3, pinned_low_bits=2, fusion_max_qubits=0, swap_mode=swap_mode)
    if dt == B.QSV_C64:
        want = want.astype(np.complex64)
        got = got.astype(np.complex64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_qv_512_thread_sections(torch, ctxs, dt):
    """chunk_bits 13 with 16 amplitudes per thread: 512-thread workgroups."""
    n = 21
    gates = W.quantum_volume(n, 8, 6)
    got, plan = run_gpu(torch, ctxs, n, gates, dt, chunk_bits=13, register_bits=4)
    assert plan.stats()["n_sections"] > 1
    assert_close(got, oracle.apply_circuit(n, gates), dt, "qv21 c13 r4")


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_qv_fusion3_dense_only(torch, ctxs, dt):
    """fusion_max_qubits 3 on Quantum Volume: SU(4) pairs sharing a qubit fuse
    into 3-qubit dense ops, so the dense-only sections run on the r = 4,
    KMAX = 3 dense-only kernel instance."""
    n = 20
    gates = W.quantum_volume(n, n, 3)
    got, plan = run_gpu(torch, ctxs, n, gates, dt, chunk_bits=12, register_bits=4,
                        pinned_low_bits=3, fusion_max_qubits=3)
    s = plan.stats()
    assert s["n_device_ops"] < s["n_gates"]
    assert_close(got, oracle.apply_circuit(n, gates), dt, "qv20 fusion 3")


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_io_phases_option(torch, ctxs, dt):
    """io_phases = 1: sections gather/scatter through an extra op-free phase
    in the coalesced map (applies when the state has >= 2^8 chunks)."""
    n = 21
    for gates in (W.quantum_volume(n, 6, 8), W.random_circuit(n, 120, 13, max_unitary_qubits=2)):
        got, plan = run_gpu(torch, ctxs, n, gates, dt, chunk_bits=12, io_phases=1)
        assert_close(got, oracle.apply_circuit(n, gates), dt, "io_phases")


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_swap_only_sections_in_place(torch, ctxs, dt):
    """SWAP-only sections: one phase, no transposition, amplitudes change
    thread (and wave) between the gather and the in-place scatter.  Bit-exact,
    on every one of several runs, with thousands of workgroups in flight."""
    n = 21
    gates = W.random_circuit(n, 40, 5, kinds=["swap"])
    psi0 = random_state(n, 7)
    if dt == B.QSV_C64:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    want = oracle.apply_circuit(n, gates, psi0)
    if dt == B.QSV_C64:
        want = want.astype(np.complex64)
    for _ in range(3):
        got, plan = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, chunk_bits=12)
        if dt == B.QSV_C64:
            got = got.astype(np.complex64)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_materialised_swaps(torch, ctxs, dt):
    n = 16
    gates = W.quantum_volume(n, 8, 5)
    psi0 = random_state(n, 5)
    want = oracle.apply_circuit(n, gates, psi0)
    got, plan = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, chunk_bits=9, register_bits=4,
                        swap_mode=B.QSV_SWAP_MATERIALIZE)
    assert plan.stats()["n_chunk_swaps"] > 0
    assert_close(got, want, dt)


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_qv_and_u3cx_midsize(torch, ctxs, dt):
    n = 20
    for gates in (W.quantum_volume(n, n, 1), W.u3_cx_layers(n, 10, 1)):
        want = oracle.apply_circuit(n, gates)
        got, _ = run_gpu(torch, ctxs, n, gates, dt)
        assert_close(got, want, dt)


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_qft_basis_closed_form(torch, ctxs, dt):
    n = 22
    x = W.random_basis_index(n, 0)
    plan = B.Plan(n, W.qft(n), dt)
    ctx = ctxs[dt]
    st = torch.empty(1 << n, dtype=tdtype(torch, dt), device="cuda")
    ctx.init_basis(st, n, x)
    ctx.apply(plan, st)
    got = st.cpu().numpy().astype(np.complex128)
    want = oracle.closed_forms.qft_basis_amplitudes(n, x, range(1 << n)) if n <= 16 else None
    ys = np.random.default_rng(0).integers(0, 1 << n, 4096)
    want = oracle.closed_forms.qft_basis_amplitudes(n, x, ys)
    tol = 1e-13 if dt == B.QSV_C128 else 2e-6
    assert np.max(np.abs(got[ys] - want)) < tol * 1
    assert abs(oracle.norm2(got) - 1.0) < (1e-12 if dt == B.QSV_C128 else 1e-5)


def test_determinism(torch, ctxs):
    n = 18
    gates = W.quantum_volume(n, n, 9)
    a, _ = run_gpu(torch, ctxs, n, gates, B.QSV_C128)
    b, _ = run_gpu(torch, ctxs, n, gates, B.QSV_C128)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_reductions(torch, ctxs, dt):
    n = 17
    ctx = ctxs[dt]
    a = random_state(n, 1) * 1.3
    b = random_state(n, 2)
    ta, tb = to_dev(torch, a, dt), to_dev(torch, b, dt)
    a_ = ta.cpu().numpy().astype(np.complex128)
    b_ = tb.cpu().numpy().astype(np.complex128)
    nrm = ctx.norm(ta, n).item()
    assert abs(nrm - oracle.norm2(a_)) < 1e-12 * nrm
    ov = ctx.overlap(ta, tb, n).cpu().numpy()
    want = oracle.overlap(a_, b_)
    assert abs(complex(ov[0], ov[1]) - want) < 1e-12
    assert abs(ov[2] - oracle.norm2(a_)) < 1e-12 * ov[2] and abs(ov[3] - oracle.norm2(b_)) < 1e-12
    terms = oracle.ring_zz_terms(n) + [(0.25, 0b101), (-1.5, 1 << (n - 1))]
    e = ctx.expval(ta, n, terms).item()
    assert abs(e - oracle.zstring_expval(a_, n, terms)) < 1e-11
    nn = ctx.normalize(ta, n).item()
    assert abs(nn - oracle.norm2(a_)) < 1e-12 * nn
    assert abs(ctx.norm(ta, n).item() - 1.0) < (1e-14 if dt == B.QSV_C128 else 1e-6)


def test_sections_prefix(torch, ctxs):
    """Checkpoint/resume: running sections [0, k) then [k, S) equals one run,
    and each prefix is a valid state of the reordered circuit prefix."""
    n = 16
    gates = W.quantum_volume(n, n, 2)
    plan = B.Plan(n, gates, B.QSV_C128, chunk_bits=8)
    S = plan.stats()["n_sections"]
    ctx = ctxs[B.QSV_C128]
    st = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    ctx.init_basis(st, n, 0)
    k = S // 2
    ctx.apply_sections(plan, st, 0, k)
    ops = plan.export()
    cut, seen = 0, 0
    for i, op in enumerate(ops):
        if op[0] == "end":
            seen += 1
            if seen == k:
                cut = i + 1
                break
    prefix_gates = [gates[op[1]] for op in ops[:cut] if op[0] == "gate"]
    want = oracle.apply_circuit(n, prefix_gates)
    assert 1 - oracle.fidelity(st.cpu().numpy(), want) < 1e-12
    ctx.apply_sections(plan, st, k, S)
    assert 1 - oracle.fidelity(st.cpu().numpy(), oracle.apply_circuit(n, gates)) < 1e-12


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_params_batch(torch, ctxs, dt):
    """Parameter-bound RY/RZ gates, several parameter sets in one launch."""
    n, layers, batch = 10, 3, 4
    tmpl = W.hardware_efficient_ansatz(n, layers)
    theta = W.ansatz_parameters(n, layers, batch, 5)
    plan = B.Plan(n, tmpl, dt, chunk_bits=7, register_bits=3)
    ctx = ctxs[dt]
    st = torch.empty(batch << n, dtype=tdtype(torch, dt), device="cuda")
    for b in range(batch):
        ctx.init_basis(st[b << n:(b + 1) << n], n, 0)
    ctx.apply_params(plan, st, torch.from_numpy(theta).cuda())
    out = st.cpu().numpy().astype(np.complex128).reshape(batch, -1)
    for b in range(batch):
        want = oracle.apply_circuit(n, oracle.bind_params(tmpl, theta[b]))
        assert_close(out[b], want, dt)


def test_empty_and_tiny(torch, ctxs):
    for n in (1, 2, 3):
        got, _ = run_gpu(torch, ctxs, n, [], B.QSV_C128, psi0=random_state(n, 0))
        assert np.allclose(got, random_state(n, 0), atol=1e-15)
    got, _ = run_gpu(torch, ctxs, 1, [W.Gate("h", (0,))], B.QSV_C128)
    assert np.allclose(got, [2 ** -0.5, 2 ** -0.5], atol=1e-15)


def test_invalid_calls(torch, ctxs):
    ctx = ctxs[B.QSV_C128]
    plan = B.Plan(10, W.ghz(10), B.QSV_C64)
    st = torch.zeros(1 << 10, dtype=torch.complex128, device="cuda")
    with pytest.raises(B.QsvError):
        ctx.apply(plan, st)  # dtype mismatch
    with pytest.raises(B.QsvError):
        ctx.init_basis(st, 10, 1 << 10)
    p2 = B.Plan(10, W.ghz(10), B.QSV_C128)
    with pytest.raises(B.QsvError):
        ctx.apply(p2, st, mode=7)


def test_large_qv_vs_oracle(torch, ctxs):
    """23 qubits at chunk 10: 8192 chunks per section, more workgroups than
    the device holds at once."""
    n = 23
    gates = W.quantum_volume(n, n, 4)
    got, plan = run_gpu(torch, ctxs, n, gates, B.QSV_C128, chunk_bits=10, register_bits=4)
    assert plan.stats()["n_sections"] > 1
    assert_close(got, oracle.apply_circuit(n, gates), B.QSV_C128, "qv23")


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_beam_and_exact_planner_plans(torch, ctxs, dt):
    """Plans of the beam-search and exact planners run on the device and match
    the oracle (the section sequence differs, the state does not)."""
    n = 20
    gates = W.quantum_volume(n, n, 5)
    psi0 = random_state(n, 5)
    want = oracle.apply_circuit(n, gates, psi0)
    got, plan = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, planner=B.QSV_PLANNER_BEAM)
    assert_close(got, want, dt, "beam")
    assert plan.stats()["n_sections"] <= B.Plan(n, gates, dt).stats()["n_sections"]
    n = 9
    gates = W.random_circuit(n, 40, 6, max_unitary_qubits=2)
    psi0 = random_state(n, 6)
    got, plan = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, planner=B.QSV_PLANNER_EXACT,
                        chunk_bits=5, register_bits=3, pinned_low_bits=1)
    assert_close(got, oracle.apply_circuit(n, gates, psi0), dt, "exact")


LDS_CASES = [
    # n, chunk_bits, fusion, seed
    (3, 3, 0, 0),
    (6, 4, 2, 1),      # 16-amplitude chunk: fewer amplitudes than threads
    (9, 7, 2, 2),
    (12, 10, 3, 3),
    (15, 12, 4, 4),
    (17, 13, 2, 5),
    (19, 11, 3, 6),
]


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
@pytest.mark.parametrize("n,c,f,seed", LDS_CASES)
def test_lds_kernel_random_circuits(torch, ctxs, dt, n, c, f, seed):
    """The LDS-resident section kernel on random circuits of every gate kind
    (SWAP relabelling, diagonal gates on local and non-local qubits, CX with local
    and non-local controls, dense gates up to 4 qubits after fusion)."""
    gates = W.random_circuit(n, 6 * n + 10, 50 + seed, max_unitary_qubits=min(3, n))
    psi0 = random_state(n, seed)
    want = oracle.apply_circuit(n, gates, psi0)
    got, plan = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, chunk_bits=c, fusion_max_qubits=f,
                        section_kernel=B.QSV_KERNEL_LDS, pinned_low_bits=min(3, c - 2))
    assert plan.stats()["register_bits"] == min(c, n)
    assert_close(got, want, dt, "lds")


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_lds_kernel_qv_and_wide(torch, ctxs, dt):
    n = 20
    gates = W.quantum_volume(n, n, 9)
    psi0 = random_state(n, 9)
    for f in (2, 3, 4):
        got, _ = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, section_kernel=B.QSV_KERNEL_LDS,
                         fusion_max_qubits=f)
        assert_close(got, oracle.apply_circuit(n, gates, psi0), dt, "lds qv f=%d" % f)
    rng = np.random.default_rng(4)
    wide = [W.Gate("unitary", tuple(int(v) for v in rng.choice(14, size=4, replace=False)), (),
                   W.haar_unitary(rng, 16)) for _ in range(5)]
    psi0 = random_state(14, 4)
    got, _ = run_gpu(torch, ctxs, 14, wide, dt, psi0=psi0, chunk_bits=10,
                     section_kernel=B.QSV_KERNEL_LDS)
    assert_close(got, oracle.apply_circuit(14, wide, psi0), dt, "lds 4-qubit unitaries")


MFMA_CASES = [
    # n, chunk_bits, fusion, seed
    (9, 9, 4, 0),      # one chunk; 5-qubit blocks fill a single tile of 16 groups
    (12, 9, 5, 1),
    (14, 10, 4, 2),
    (16, 12, 5, 3),
    (18, 13, 5, 4),
    (20, 11, 4, 5),
]


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
@pytest.mark.parametrize("n,c,f,seed", MFMA_CASES)
def test_mfma_fused_blocks(torch, ctxs, dt, n, c, f, seed):
    """Matrix-core section path: in-section gates fused into blocks of up to f
    qubits (commuting gates gathered across the section) and applied as complex
    matrix products with MFMA; random circuits of every gate kind (diagonal and
    CX with non-local sources stay separate ops) followed by QV layers."""
    gates = (W.random_circuit(n, 6 * n + 10, 70 + seed, max_unitary_qubits=3)
             + W.quantum_volume(n, 6, 80 + seed))
    psi0 = random_state(n, seed)
    want = oracle.apply_circuit(n, gates, psi0)
    got, plan = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, chunk_bits=c, fusion_max_qubits=f,
                        section_kernel=B.QSV_KERNEL_MFMA, pinned_low_bits=min(3, c - 5))
    assert plan.stats()["fusion_max_qubits"] == f
    assert_close(got, want, dt, "mfma f=%d" % f)


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_mfma_wide_unitaries_and_qv(torch, ctxs, dt):
    """Unfused 4- and 5-qubit Haar unitaries on scattered qubits, and a QV
    circuit at fusion 4 and 5, through the matrix-core path."""
    rng = np.random.default_rng(12)
    n = 15
    wide = [W.Gate("unitary", tuple(int(v) for v in rng.choice(n, size=k, replace=False)), (),
                   W.haar_unitary(rng, 1 << k)) for k in (4, 5, 5, 4, 5, 3, 5)]
    psi0 = random_state(n, 12)
    got, _ = run_gpu(torch, ctxs, n, wide, dt, psi0=psi0, chunk_bits=11, fusion_max_qubits=0,
                     section_kernel=B.QSV_KERNEL_MFMA)
    assert_close(got, oracle.apply_circuit(n, wide, psi0), dt, "mfma wide unitaries")
    n = 20
    gates = W.quantum_volume(n, n, 13)
    psi0 = random_state(n, 13)
    want = oracle.apply_circuit(n, gates, psi0)
    for f in (4, 5):
        got, _ = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, chunk_bits=12 if dt == B.QSV_C128 else 13,
                         fusion_max_qubits=f, section_kernel=B.QSV_KERNEL_MFMA)
        assert_close(got, want, dt, "mfma qv f=%d" % f)


PAIRED_CASES = [
    # n, chunk_bits, seed
    (6, 4, 0), (9, 6, 1), (12, 8, 2), (16, 12, 3), (18, 13, 4), (20, 11, 5),
]


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
@pytest.mark.parametrize("n,c,seed", PAIRED_CASES)
def test_paired_sections_qv(torch, ctxs, dt, n, c, seed):
    """Paired phases (two fused gate pairs at fixed register positions) on
    Quantum-Volume circuits, several phases per section and one-pair phases."""
    gates = W.quantum_volume(n, n, 30 + seed)
    psi0 = random_state(n, seed)
    want = oracle.apply_circuit(n, gates, psi0)
    for planner in (B.QSV_PLANNER_DEFAULT, B.QSV_PLANNER_BEAM):
        got, plan = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, chunk_bits=c,
                            section_kernel=B.QSV_KERNEL_PAIRED, planner=planner,
                            pinned_low_bits=min(3, c - 4))
        assert plan.stats()["register_bits"] == 4
        assert_close(got, want, dt, "paired planner %d" % planner)


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_paired_mixed_sections(torch, ctxs, dt):
    """Circuits whose sections mix 2-qubit dense gates with other kinds: the
    eligible sections run paired phases, the others the general register phases
    (same plan, both kernels), and the result matches the oracle."""
    n = 16
    rng = np.random.default_rng(8)
    gates = []
    for layer in range(10):
        perm = rng.permutation(n)
        for i in range(n // 2):
            gates.append(W.Gate("unitary", (int(perm[2 * i]), int(perm[2 * i + 1])), (),
                                W.haar_su(rng, 4)))
        if layer % 3 == 2:
            gates += W.random_circuit(n, 12, 100 + layer, max_unitary_qubits=3)
    psi0 = random_state(n, 8)
    got, plan = run_gpu(torch, ctxs, n, gates, dt, psi0=psi0, chunk_bits=10,
                        section_kernel=B.QSV_KERNEL_PAIRED)
    assert_close(got, oracle.apply_circuit(n, gates, psi0), dt, "paired mixed")
    # the same plan through the batch kernel (general phases execute paired tables)
    if dt == B.QSV_C64:
        plans = [B.Plan(n, gates, dt, chunk_bits=11, section_kernel=B.QSV_KERNEL_PAIRED)]
        st = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
        ctxs[dt].batch_run(plans, [0], st)
        torch.cuda.synchronize()
        want = oracle.apply_circuit(n, gates)
        got = st.cpu().numpy().astype(np.complex128)
        assert 1.0 - oracle.fidelity(got, want) < 1e-5
