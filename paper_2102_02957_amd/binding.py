"""ctypes binding of the C ABI in include/qsv.h (argument marshalling only).

Every computation runs in libqsv.so's HIP kernels; this module converts gate
lists to ``qsv_gate`` arrays, passes device pointers of torch tensors and the
current HIP stream, and turns status codes into exceptions.  If the shared
library is missing the import of ``lib()`` raises: there is no fallback.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqsv.so")

QSV_C64, QSV_C128 = 1, 2
QSV_SWAP_REMAP, QSV_SWAP_MATERIALIZE = 0, 1
QSV_MODE_BLOCKED, QSV_MODE_PER_GATE = 0, 1
QSV_OP_BEGIN, QSV_OP_END, QSV_OP_CHUNK_SWAP, QSV_OP_GATE = 1, 2, 3, 4
QSV_PLANNER_DEFAULT, QSV_PLANNER_GREEDY, QSV_PLANNER_BEAM, QSV_PLANNER_EXACT = 0, 1, 2, 3
QSV_KERNEL_REGISTERS, QSV_KERNEL_LDS, QSV_KERNEL_PAIRED, QSV_KERNEL_MFMA = 0, 1, 2, 3

KINDS = {k: i + 1 for i, k in enumerate(
    ["h", "x", "y", "z", "s", "sdg", "t", "tdg", "rx", "ry", "rz", "p", "u3",
     "cx", "cz", "cp", "swap", "unitary",
     "amp_damp", "phase_damp", "depolarize", "kraus"])}

STATUS = {0: "QSV_OK", -1: "QSV_E_INVALID", -2: "QSV_E_NOMEM", -3: "QSV_E_HIP",
          -4: "QSV_E_UNSUPPORTED", -5: "QSV_E_NUMERIC", -6: "QSV_E_STATE"}


class QsvError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nq", ctypes.c_int32), ("q", ctypes.c_int32 * 5),
                ("param", ctypes.c_int32), ("p", ctypes.c_double * 3),
                ("m", ctypes.POINTER(ctypes.c_double))]


class Options(ctypes.Structure):
    _fields_ = [("chunk_bits", ctypes.c_int32), ("pinned_low_bits", ctypes.c_int32),
                ("fusion_max_qubits", ctypes.c_int32), ("swap_mode", ctypes.c_int32),
                ("diag_free", ctypes.c_int32), ("register_bits", ctypes.c_int32),
                ("io_phases", ctypes.c_int32), ("planner", ctypes.c_int32),
                ("section_kernel", ctypes.c_int32)]


class PlanStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dtype", ctypes.c_int32), ("chunk_bits", ctypes.c_int32),
                ("register_bits", ctypes.c_int32), ("pinned_low_bits", ctypes.c_int32),
                ("fusion_max_qubits", ctypes.c_int32), ("swap_mode", ctypes.c_int32),
                ("diag_free", ctypes.c_int32), ("n_gates", ctypes.c_int64),
                ("n_sections", ctypes.c_int64), ("n_chunk_swaps", ctypes.c_int64),
                ("n_phases", ctypes.c_int64), ("n_device_ops", ctypes.c_int64),
                ("n_params", ctypes.c_int64), ("section_flops", ctypes.c_double),
                ("final_perm", ctypes.c_int32 * 64)]


class Op(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int32), ("gate", ctypes.c_int32), ("nq", ctypes.c_int32),
                ("q", ctypes.c_int32 * 5), ("mask", ctypes.c_uint64)]


class ZTerm(ctypes.Structure):
    _fields_ = [("coeff", ctypes.c_double), ("zmask", ctypes.c_uint64)]


EXPORTED = [
    "qsv_default_options", "qsv_plan_blocks", "qsv_plan_destroy", "qsv_plan_get_stats",
    "qsv_plan_export", "qsv_create", "qsv_destroy", "qsv_last_error", "qsv_init_basis",
    "qsv_apply_circuit", "qsv_apply_sections", "qsv_apply_params", "qsv_norm", "qsv_overlap",
    "qsv_expval", "qsv_normalize", "qsv_copy", "qsv_adjoint_grad", "qsv_batch_run",
    "qsv_timing_enable", "qsv_timing_read", "qsv_autotune", "qsv_autotune_batch",
    "qsv_reserve", "qsv_overlap_noalloc", "qsv_plan_density", "qsv_dm_trace", "qsv_dm_expval",
    "qsv_autotune_adjoint", "qsv_apply_host", "qsv_plan_stream_bits",
]

_lib = None


def lib():
    """Load libqsv.so (built in-tree by ``paper_2102_02957_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqsv.so not built: run `python -m paper_2102_02957_amd.build` "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, I, U64, SZ, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double
    sigs = {
        "qsv_default_options": (I, [I, ctypes.POINTER(Options)]),
        "qsv_plan_blocks": (I, [ctypes.POINTER(Options), I, I, ctypes.POINTER(Gate), SZ,
                                ctypes.POINTER(P)]),
        "qsv_plan_destroy": (None, [P]),
        "qsv_plan_get_stats": (I, [P, ctypes.POINTER(PlanStats)]),
        "qsv_plan_export": (I, [P, ctypes.POINTER(Op), SZ, ctypes.POINTER(SZ)]),
        "qsv_create": (I, [ctypes.POINTER(P), I, I]),
        "qsv_destroy": (None, [P]),
        "qsv_last_error": (ctypes.c_char_p, []),
        "qsv_init_basis": (I, [P, P, I, U64, P]),
        "qsv_apply_circuit": (I, [P, P, P, I, I, P]),
        "qsv_apply_sections": (I, [P, P, P, I, ctypes.c_int64, ctypes.c_int64, P]),
        "qsv_apply_params": (I, [P, P, P, I, I, P, P]),
        "qsv_norm": (I, [P, P, I, P, P]),
        "qsv_overlap": (I, [P, P, P, I, P, P]),
        "qsv_expval": (I, [P, P, I, ctypes.POINTER(ZTerm), SZ, P, P]),
        "qsv_normalize": (I, [P, P, I, P, P]),
        "qsv_copy": (I, [P, P, P, I, P]),
        "qsv_adjoint_grad": (I, [P, P, ctypes.POINTER(ZTerm), SZ, P, I, P, P, P, P, P]),
        "qsv_batch_run": (I, [P, I, ctypes.POINTER(P), ctypes.POINTER(U64), P, P, P]),
        "qsv_reserve": (I, [P, P, I, I, P]),
        "qsv_apply_host": (I, [P, P, P, I, SZ, ctypes.c_int64, ctypes.c_int64, P]),
        "qsv_plan_stream_bits": (I, [P, I, ctypes.POINTER(U64)]),
        "qsv_plan_density": (I, [ctypes.POINTER(Options), I, I, ctypes.POINTER(Gate), SZ,
                                 ctypes.POINTER(P)]),
        "qsv_dm_trace": (I, [P, P, I, P, P]),
        "qsv_dm_expval": (I, [P, P, I, ctypes.POINTER(ZTerm), SZ, P, P]),
        "qsv_overlap_noalloc": (I, [P, P, P, I, P, P]),
        "qsv_timing_enable": (I, [P, I]),
        "qsv_timing_read": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_int64), I]),
        "qsv_autotune": (I, [P, I, I, ctypes.POINTER(Gate), SZ, ctypes.POINTER(Options), I, P, I, I,
                             I, P, ctypes.POINTER(I), ctypes.POINTER(D)]),
        "qsv_autotune_adjoint": (I, [P, I, I, ctypes.POINTER(Gate), SZ, ctypes.POINTER(ZTerm), SZ, P,
                                     I, P, P, P, P, ctypes.POINTER(Options), I, I, P,
                                     ctypes.POINTER(I), ctypes.POINTER(D)]),
        "qsv_autotune_batch": (I, [P, I, I, ctypes.POINTER(I), ctypes.POINTER(ctypes.POINTER(Gate)),
                                   ctypes.POINTER(SZ), ctypes.POINTER(U64), ctypes.POINTER(Options),
                                   I, P, P, I, P, ctypes.POINTER(I), ctypes.POINTER(D)]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise QsvError(rc, lib().qsv_last_error().decode(errors="replace"))


def default_options(dtype):
    o = Options()
    _check(lib().qsv_default_options(dtype, ctypes.byref(o)))
    return o


def make_options(dtype, **kw):
    o = default_options(dtype)
    for k, v in kw.items():
        if v is None:
            continue
        if not hasattr(o, k):
            raise TypeError("unknown option %r" % k)
        setattr(o, k, int(v))
    return o


def gates_to_c(gates):
    """Convert gate tuples (kind, qubits, params, matrix, pidx) to a qsv_gate array.
    Returns (array, keepalive)."""
    arr = (Gate * max(1, len(gates)))()
    keep = []
    for i, g in enumerate(gates):
        kind, qubits, params, matrix, pidx = g[0], g[1], g[2], g[3], (g[4] if len(g) > 4 else -1)
        c = arr[i]
        if kind not in KINDS:
            raise ValueError("unknown gate kind %r" % (kind,))
        c.kind = KINDS[kind]
        c.nq = len(qubits)
        for j, q in enumerate(qubits):
            c.q[j] = int(q)
        c.param = -1 if pidx is None else int(pidx)
        for j, v in enumerate(params):
            c.p[j] = float(v)
        if kind in ("unitary", "kraus") and matrix is not None:
            m = np.ascontiguousarray(np.asarray(matrix, dtype=np.complex128))
            if kind == "kraus":
                c.param = int(m.shape[0])      # number of Kraus operators
            buf = m.view(np.float64)
            keep.append(buf)
            c.m = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            c.m = None
    return arr, keep


class Plan:
    """A cache-blocked plan (host object; see qsv_plan_blocks)."""

    def __init__(self, n, gates, dtype=QSV_C128, **options):
        self.n = int(n)
        self.dtype = dtype
        self.gates = list(gates)
        opt = make_options(dtype, **options)
        arr, keep = gates_to_c(self.gates)
        h = ctypes.c_void_p()
        _check(lib().qsv_plan_blocks(ctypes.byref(opt), dtype, self.n, arr, len(self.gates),
                                     ctypes.byref(h)))
        self._h = h
        del keep

    @classmethod
    def density(cls, n, gates, dtype=QSV_C128, **options):
        """qsv_plan_density: the 2n-qubit plan of an n-qubit circuit with channels
        acting on its density matrix (rho[i][j] at index i | j << n)."""
        self = cls.__new__(cls)
        self.n = 2 * int(n)
        self.n_density = int(n)
        self.dtype = dtype
        self.gates = list(gates)
        opt = make_options(dtype, **options)
        arr, keep = gates_to_c(self.gates)
        h = ctypes.c_void_p()
        _check(lib().qsv_plan_density(ctypes.byref(opt), dtype, int(n), arr, len(self.gates),
                                      ctypes.byref(h)))
        self._h = h
        del keep
        return self

    @property
    def handle(self):
        return self._h

    def stats(self):
        s = PlanStats()
        _check(lib().qsv_plan_get_stats(self._h, ctypes.byref(s)))
        d = {f: getattr(s, f) for f, _ in PlanStats._fields_ if f != "final_perm"}
        d["final_perm"] = [s.final_perm[q] for q in range(self.n)]
        return d

    def stream_bits(self, o):
        """qsv_plan_stream_bits: the cut bits of every section for o slice bits."""
        S = self.stats()["n_sections"]
        out = (ctypes.c_uint64 * S)()
        _check(lib().qsv_plan_stream_bits(self._h, int(o), out))
        return [int(v) for v in out]

    def export(self):
        """The transpiled op list in the oracle's plan format."""
        need = ctypes.c_size_t()
        _check(lib().qsv_plan_export(self._h, None, 0, ctypes.byref(need)))
        ops = (Op * max(1, need.value))()
        _check(lib().qsv_plan_export(self._h, ops, need.value, ctypes.byref(need)))
        out = []
        for o in ops[:need.value]:
            if o.tag == QSV_OP_BEGIN:
                out.append(("begin", int(o.mask)))
            elif o.tag == QSV_OP_END:
                out.append(("end",))
            elif o.tag == QSV_OP_CHUNK_SWAP:
                out.append(("swap", o.q[0], o.q[1]))
            else:
                out.append(("gate", o.gate, tuple(o.q[j] for j in range(o.nq))))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.qsv_plan_destroy(h)
            self._h = None


def _torch():
    import torch
    return torch


def dtype_of(t):
    torch = _torch()
    if t.dtype == torch.complex128:
        return QSV_C128
    if t.dtype == torch.complex64:
        return QSV_C64
    raise TypeError("state must be complex64 or complex128, got %s" % t.dtype)


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_state(t, n, batch=1, dtype=None):
    """Host-side checks the C ABI cannot make (it sees pointers, not sizes)."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("state must be a contiguous device tensor")
    if dtype is not None and dtype_of(t) != dtype:
        raise ValueError("state dtype %s does not match the context's %s"
                         % (t.dtype, "complex128" if dtype == QSV_C128 else "complex64"))
    if t.numel() != (batch << n):
        raise ValueError("state must hold %d x 2^%d amplitudes" % (batch, n))


def _check_f64(t, shape, what):
    torch = _torch()
    if (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()
            or tuple(t.shape) != tuple(shape)):
        raise ValueError("%s must be a contiguous float64 device tensor of shape %s"
                         % (what, tuple(shape)))


class Context:
    """A device context (qsv_create) for one dtype."""

    def __init__(self, dtype=QSV_C128, device=0):
        self.dtype = dtype
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().qsv_create(ctypes.byref(h), int(device), int(dtype)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.qsv_destroy(h)
            self._h = None

    def init_basis(self, state, n, basis=0, stream=None):
        _check_state(state, n, dtype=self.dtype)
        _check(lib().qsv_init_basis(self._h, _ptr(state), n, int(basis), _stream(stream)))

    def apply(self, plan, state, mode=QSV_MODE_BLOCKED, stream=None):
        _check_state(state, plan.n, dtype=self.dtype)
        _check(lib().qsv_apply_circuit(self._h, plan.handle, _ptr(state), plan.n, int(mode),
                                       _stream(stream)))

    def apply_sections(self, plan, state, s0, s1, stream=None):
        _check_state(state, plan.n, dtype=self.dtype)
        _check(lib().qsv_apply_sections(self._h, plan.handle, _ptr(state), plan.n, int(s0),
                                        int(s1), _stream(stream)))

    def reserve(self, plan=None, n=None, batch=1, stream=None):
        """qsv_reserve: size the workspaces (and upload the plan) so that later
        calls allocate nothing and can be captured into a graph."""
        n = plan.n if plan is not None else int(n)
        _check(lib().qsv_reserve(self._h, plan.handle if plan is not None else None, n,
                                 int(batch), _stream(stream)))

    def apply_host(self, plan, host_state, hbm_budget, s0=0, s1=None, stream=None):
        """qsv_apply_host: sections [s0, s1) on a pinned host tensor (torch
        pin_memory=True), streamed through at most `hbm_budget` bytes of HBM."""
        torch = _torch()
        if host_state.is_cuda or not host_state.is_contiguous() or not host_state.is_pinned():
            raise ValueError("host_state must be a contiguous pinned host tensor")
        if dtype_of(host_state) != self.dtype or host_state.numel() != (1 << plan.n):
            raise ValueError("host_state must hold 2^n amplitudes of the context's dtype")
        s1 = plan.stats()["n_sections"] if s1 is None else s1
        _check(lib().qsv_apply_host(self._h, plan.handle, ctypes.c_void_p(host_state.data_ptr()),
                                    plan.n, int(hbm_budget), int(s0), int(s1), _stream(stream)))

    def apply_params(self, plan, states, params, stream=None):
        batch = params.shape[0] if params.dim() == 2 else -1
        _check_f64(params, (batch, plan.stats()["n_params"]), "params")
        _check_state(states, plan.n, batch, dtype=self.dtype)
        _check(lib().qsv_apply_params(self._h, plan.handle, _ptr(states), plan.n, int(batch),
                                      _ptr(params), _stream(stream)))

    def norm(self, state, n, out=None, stream=None):
        torch = _torch()
        _check_state(state, n, dtype=self.dtype)
        out = torch.empty(1, dtype=torch.float64, device=state.device) if out is None else out
        _check_f64(out, (1,), "out")
        _check(lib().qsv_norm(self._h, _ptr(state), n, _ptr(out), _stream(stream)))
        return out

    def overlap(self, a, b, n, out=None, stream=None):
        torch = _torch()
        _check_state(a, n, dtype=self.dtype)
        _check_state(b, n, dtype=self.dtype)
        out = torch.empty(4, dtype=torch.float64, device=a.device) if out is None else out
        _check_f64(out, (4,), "out")
        _check(lib().qsv_overlap(self._h, _ptr(a), _ptr(b), n, _ptr(out), _stream(stream)))
        return out

    def overlap_noalloc(self, a, b, n, out, stream=None):
        """qsv_overlap_noalloc: the caller supplies `out` (float64[4] on the device)."""
        _check_state(a, n, dtype=self.dtype)
        _check_state(b, n, dtype=self.dtype)
        _check_f64(out, (4,), "out")
        _check(lib().qsv_overlap_noalloc(self._h, _ptr(a), _ptr(b), n, _ptr(out), _stream(stream)))
        return out

    def expval(self, state, n, terms, out=None, stream=None):
        torch = _torch()
        _check_state(state, n, dtype=self.dtype)
        arr = (ZTerm * len(terms))()
        for i, (c, m) in enumerate(terms):
            arr[i].coeff = float(c)
            arr[i].zmask = int(m)
        out = torch.empty(1, dtype=torch.float64, device=state.device) if out is None else out
        _check_f64(out, (1,), "out")
        _check(lib().qsv_expval(self._h, _ptr(state), n, arr, len(terms), _ptr(out),
                                _stream(stream)))
        return out

    def dm_init_basis(self, rho, n, basis=0, stream=None):
        """rho <- |basis><basis| for an n-qubit density matrix (2^(2n) amplitudes)."""
        self.init_basis(rho, 2 * n, int(basis) | (int(basis) << n), stream)

    def dm_trace(self, rho, n, out=None, stream=None):
        torch = _torch()
        _check_state(rho, 2 * n, dtype=self.dtype)
        out = torch.empty(1, dtype=torch.float64, device=rho.device) if out is None else out
        _check_f64(out, (1,), "out")
        _check(lib().qsv_dm_trace(self._h, _ptr(rho), n, _ptr(out), _stream(stream)))
        return out

    def dm_expval(self, rho, n, terms, out=None, stream=None):
        torch = _torch()
        _check_state(rho, 2 * n, dtype=self.dtype)
        arr = (ZTerm * len(terms))()
        for i, (c, m) in enumerate(terms):
            arr[i].coeff = float(c)
            arr[i].zmask = int(m)
        out = torch.empty(1, dtype=torch.float64, device=rho.device) if out is None else out
        _check_f64(out, (1,), "out")
        _check(lib().qsv_dm_expval(self._h, _ptr(rho), n, arr, len(terms), _ptr(out),
                                   _stream(stream)))
        return out

    def normalize(self, state, n, out=None, stream=None):
        torch = _torch()
        _check_state(state, n, dtype=self.dtype)
        out = torch.empty(1, dtype=torch.float64, device=state.device) if out is None else out
        _check_f64(out, (1,), "out")
        _check(lib().qsv_normalize(self._h, _ptr(state), n, _ptr(out), _stream(stream)))
        return out

    def copy(self, dst, src, n, stream=None):
        _check_state(dst, n, dtype=self.dtype)
        _check_state(src, n, dtype=self.dtype)
        _check(lib().qsv_copy(self._h, _ptr(dst), _ptr(src), n, _stream(stream)))

    def timing(self, enable):
        _check(lib().qsv_timing_enable(self._h, 1 if enable else 0))

    def timing_read(self, which=0, reset=True):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(lib().qsv_timing_read(self._h, int(which), ctypes.byref(ms), ctypes.byref(cnt),
                                     1 if reset else 0))
        return ms.value, cnt.value


def _batch_run(self, plans, offsets, states, norms=None, stream=None):
    """qsv_batch_run: plans[b] applied to the state at states[offsets[b]:], all
    initialised to |0>, FP64-renormalised; returns the pre-normalisation norms."""
    torch = _torch()
    count = len(plans)
    if not states.is_cuda or not states.is_contiguous():
        raise ValueError("states must be a contiguous device tensor")
    if dtype_of(states) != self.dtype:
        raise ValueError("states dtype does not match the context")
    if len(offsets) != count:
        raise ValueError("one offset per plan")
    for p, o in zip(plans, offsets):
        if o + (1 << p.n) > states.numel():
            raise ValueError("state of a plan runs past the buffer")
    arr = (ctypes.c_void_p * count)(*[p.handle.value for p in plans])
    offs = (ctypes.c_uint64 * count)(*[int(o) for o in offsets])
    norms = torch.empty(count, dtype=torch.float64, device=states.device) if norms is None else norms
    _check_f64(norms, (count,), "norms")
    _check(lib().qsv_batch_run(self._h, count, arr, offs, _ptr(states), _ptr(norms), _stream(stream)))
    return norms


def _adjoint_grad(self, plan, terms, params, psi, lam, energy=None, grad=None, stream=None):
    """qsv_adjoint_grad: energies [B] and gradients [B, P] of <psi|H|psi>."""
    torch = _torch()
    batch = params.shape[0] if params.dim() == 2 else -1
    nparams = plan.stats()["n_params"]
    _check_f64(params, (batch, nparams), "params")
    _check_state(psi, plan.n, batch, dtype=self.dtype)
    _check_state(lam, plan.n, batch, dtype=self.dtype)
    arr = (ZTerm * len(terms))()
    for i, (c, m) in enumerate(terms):
        arr[i].coeff = float(c)
        arr[i].zmask = int(m)
    energy = torch.empty(batch, dtype=torch.float64, device=psi.device) if energy is None else energy
    grad = torch.empty(batch, max(1, nparams), dtype=torch.float64, device=psi.device) if grad is None else grad
    _check_f64(energy, (batch,), "energy")
    _check_f64(grad, (batch, max(1, nparams)), "grad")
    _check(lib().qsv_adjoint_grad(self._h, plan.handle, arr, len(terms), _ptr(params), int(batch),
                                  _ptr(psi), _ptr(lam), _ptr(energy), _ptr(grad), _stream(stream)))
    return energy, grad[:, :nparams]


Context.batch_run = _batch_run
Context.adjoint_grad = _adjoint_grad


def adjoint_energy_function():
    """A torch.autograd.Function whose forward returns E_b for params [B, P]
    (one qsv_adjoint_grad call computes E and dE/dtheta) and whose backward
    returns gE[:, None] * dE/dtheta."""
    torch = _torch()

    class AdjointEnergy(torch.autograd.Function):
        @staticmethod
        def forward(fctx, params, qctx, plan, terms):
            p = params.detach().contiguous()
            batch = p.shape[0]
            dt = torch.complex128 if plan.dtype == QSV_C128 else torch.complex64
            psi = torch.empty(batch << plan.n, dtype=dt, device=p.device)
            lam = torch.empty_like(psi)
            e, g = qctx.adjoint_grad(plan, terms, p, psi, lam)
            fctx.save_for_backward(g)
            return e

        @staticmethod
        def backward(fctx, ge):
            (g,) = fctx.saved_tensors
            return ge[:, None] * g, None, None, None

    return AdjointEnergy


def default_candidates(dtype, n):
    """A small grid around the defaults: chunk bits, pinned low bits, fusion width."""
    base = default_options(dtype)
    out = []
    for dc in (-1, 0):
        for L in (2, 3, 4):
            for f in (0, 2):
                c = min(base.chunk_bits + dc, n)
                out.append(dict(chunk_bits=c, pinned_low_bits=min(L, max(0, c - 2)),
                                fusion_max_qubits=f, register_bits=min(base.register_bits, c)))
    return out


def state_candidates(dtype, n):
    """Bounded grid for one large state: chunk bits c and register bits r around the
    defaults (within the kernels' thread limits), pinned low bits L, fusion width f,
    and the schedule options io_phases and the planner (section sequence)."""
    base = default_options(dtype)
    out = []
    for dc in (-1, 0):
        c = min(base.chunk_bits + dc, n)
        for r in (base.register_bits - 1, base.register_bits):
            if r < 1 or c - r > (9 if r <= 4 else 8):
                continue
            for L in (base.pinned_low_bits, base.pinned_low_bits + 1):
                out.append(dict(chunk_bits=c, register_bits=r, pinned_low_bits=min(L, c - 2),
                                fusion_max_qubits=2, io_phases=0))
    out.append(dict(chunk_bits=min(base.chunk_bits, n), register_bits=base.register_bits,
                    pinned_low_bits=base.pinned_low_bits, fusion_max_qubits=3, io_phases=0))
    out.append(dict(chunk_bits=min(base.chunk_bits, n), register_bits=base.register_bits,
                    pinned_low_bits=base.pinned_low_bits, fusion_max_qubits=2, io_phases=1))
    # section schedule: the beam-search planner on the default shape
    out.append(dict(chunk_bits=min(base.chunk_bits, n), register_bits=base.register_bits,
                    pinned_low_bits=base.pinned_low_bits, fusion_max_qubits=2, io_phases=0,
                    planner=QSV_PLANNER_BEAM))
    # paired phases (fixed register positions), default and beam planners, and the
    # beam planner with one more pinned low bit (longer contiguous runs, more sections)
    for c in sorted({min(base.chunk_bits, n), min(base.chunk_bits - 1, n)}):
        for pl in (QSV_PLANNER_DEFAULT, QSV_PLANNER_BEAM):
            out.append(dict(chunk_bits=c, register_bits=4, pinned_low_bits=min(3, c - 4),
                            fusion_max_qubits=2, io_phases=0, planner=pl,
                            section_kernel=QSV_KERNEL_PAIRED))
    c = min(base.chunk_bits, n)
    out.append(dict(chunk_bits=c, register_bits=4, pinned_low_bits=min(4, c - 4),
                    fusion_max_qubits=2, io_phases=0, planner=QSV_PLANNER_BEAM,
                    section_kernel=QSV_KERNEL_PAIRED))
    # fused 4-qubit blocks on the matrix cores (LDS-resident chunk)
    c = min(base.chunk_bits, n)
    if c >= 9:
        out.append(dict(chunk_bits=c, pinned_low_bits=min(base.pinned_low_bits, c - 5),
                        fusion_max_qubits=4, io_phases=0, planner=QSV_PLANNER_BEAM,
                        section_kernel=QSV_KERNEL_MFMA))
    return out


def adjoint_candidates(dtype, n):
    """Grid for the adjoint sweep: chunk and register bits (fusion of at most 2
    qubits, which the reverse sweep requires)."""
    out = []
    for c in (10, 11, 12):
        for r in (3, 4):
            if c > n or c - r > 8 or (dtype == QSV_C128 and r > 4):
                continue
            out.append(dict(chunk_bits=c, register_bits=r, fusion_max_qubits=2))
    return out


def batch_candidates(dtype):
    """Grid for qsv_batch_run: chunk bits, register bits and fusion width (each
    candidate plans every trajectory and captures its own graph, so the grid is short)."""
    if dtype == QSV_C64:
        return [dict(chunk_bits=11, register_bits=4, fusion_max_qubits=2),
                dict(chunk_bits=12, register_bits=4, fusion_max_qubits=2),
                dict(chunk_bits=12, register_bits=4, fusion_max_qubits=3),
                dict(chunk_bits=13, register_bits=5, fusion_max_qubits=2)]
    return [dict(chunk_bits=10, register_bits=3, fusion_max_qubits=2),
            dict(chunk_bits=11, register_bits=3, fusion_max_qubits=2),
            dict(chunk_bits=12, register_bits=4, fusion_max_qubits=2)]


def _options_array(dtype, cands):
    arr = (Options * len(cands))()
    for i, kw in enumerate(cands):
        arr[i] = make_options(dtype, **kw)
    return arr


def _autotune(self, n, gates, candidates=None, reps=2, scratch=None, stream=None, max_sections=0,
              refine=0):
    """qsv_autotune: returns (best option dict, per-candidate ms).  max_sections > 0
    times only that many leading sections per candidate and scales by its section
    count; refine > 0 re-times that many of the best estimates on whole applies."""
    torch = _torch()
    cands = candidates or default_candidates(self.dtype, n)
    arr = _options_array(self.dtype, cands)
    g, keep = gates_to_c(gates)
    tdt = torch.complex128 if self.dtype == QSV_C128 else torch.complex64
    st = torch.empty(1 << n, dtype=tdt, device="cuda") if scratch is None else scratch
    best = ctypes.c_int()
    ms = (ctypes.c_double * len(cands))()
    _check(lib().qsv_autotune(self._h, self.dtype, n, g, len(gates), arr, len(cands), _ptr(st),
                              int(reps), int(max_sections), int(refine), _stream(stream),
                              ctypes.byref(best), ms))
    del keep
    return cands[best.value], list(ms)


def _autotune_batch(self, circuits, offsets, states, candidates=None, reps=2, stream=None):
    """qsv_autotune_batch over (n, gates) circuits packed at `offsets` in `states`."""
    torch = _torch()
    cands = candidates or [c for c in default_candidates(self.dtype, 64) if c["chunk_bits"] <= 64]
    arr = _options_array(self.dtype, cands)
    count = len(circuits)
    ns = (ctypes.c_int * count)(*[n for n, _ in circuits])
    gl, keep, ngs = [], [], (ctypes.c_size_t * count)()
    for i, (_, gates) in enumerate(circuits):
        g, k = gates_to_c(gates)
        gl.append(g)
        keep.append(k)
        ngs[i] = len(gates)
    gp = (ctypes.POINTER(Gate) * count)(*[ctypes.cast(g, ctypes.POINTER(Gate)) for g in gl])
    offs = (ctypes.c_uint64 * count)(*[int(o) for o in offsets])
    norms = torch.empty(count, dtype=torch.float64, device=states.device)
    best = ctypes.c_int()
    ms = (ctypes.c_double * len(cands))()
    _check(lib().qsv_autotune_batch(self._h, self.dtype, count, ns, gp, ngs, offs, arr, len(cands),
                                    _ptr(states), _ptr(norms), int(reps), _stream(stream),
                                    ctypes.byref(best), ms))
    del keep, gl
    return cands[best.value], list(ms)


def _autotune_adjoint(self, n, gates, terms, params, psi, lam, candidates=None, reps=1,
                      stream=None):
    """qsv_autotune_adjoint: (best option dict, per-candidate ms per gradient call)."""
    torch = _torch()
    cands = candidates or adjoint_candidates(self.dtype, n)
    arr = _options_array(self.dtype, cands)
    g, keep = gates_to_c(gates)
    batch = params.shape[0]
    nparams = max([int(x[4]) for x in gates if len(x) > 4 and x[4] is not None] + [-1]) + 1
    _check_f64(params, (batch, nparams), "params")
    _check_state(psi, n, batch, dtype=self.dtype)
    _check_state(lam, n, batch, dtype=self.dtype)
    t = (ZTerm * len(terms))()
    for i, (c, m) in enumerate(terms):
        t[i].coeff = float(c)
        t[i].zmask = int(m)
    energy = torch.empty(batch, dtype=torch.float64, device=psi.device)
    grad = torch.empty(batch, max(1, nparams), dtype=torch.float64, device=psi.device)
    best = ctypes.c_int()
    ms = (ctypes.c_double * len(cands))()
    _check(lib().qsv_autotune_adjoint(self._h, self.dtype, n, g, len(gates), t, len(terms),
                                      _ptr(params), int(batch), _ptr(psi), _ptr(lam), _ptr(energy),
                                      _ptr(grad), arr, len(cands), int(reps), _stream(stream),
                                      ctypes.byref(best), ms))
    del keep
    return cands[best.value], list(ms)


Context.autotune = _autotune
Context.autotune_batch = _autotune_batch
Context.autotune_adjoint = _autotune_adjoint


class AutotuneCache:
    """Tuning results in a JSON file, keyed by (GPU architecture, dtype, n, circuit
    class): {key: {"chosen": options, "candidates": [options...], "ms": [...]}}.
    The file is read once and rewritten after every new entry."""

    def __init__(self, path=None):
        self.path = path or os.environ.get("QSV_AUTOTUNE_CACHE") or os.path.join(
            os.path.expanduser("~"), ".cache", "qsv", "autotune.json")
        self.data = {}
        if os.path.exists(self.path):
            import json
            try:
                with open(self.path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    @staticmethod
    def key(arch, dtype, n, circuit_class):
        return "%s|%s|n=%d|%s" % (arch, "c128" if dtype == QSV_C128 else "c64", int(n),
                                  circuit_class)

    def get(self, key):
        return self.data.get(key)

    def put(self, key, chosen, candidates, ms):
        import json
        self.data[key] = {"chosen": dict(chosen), "candidates": [dict(c) for c in candidates],
                          "ms": [None if m == float("inf") else float(m) for m in ms]}
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def tune(self, key, run):
        """Cached result for `key`, else run() -> (chosen, candidates, ms), stored.
        Returns (entry, hit)."""
        hit = self.get(key)
        if hit is not None:
            return hit, True
        chosen, cands, ms = run()
        self.put(key, chosen, cands, ms)
        return self.get(key), False
