"""Reference oracle for cache-blocked state-vector gate application.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct CPU
implementation (NumPy, complex128 / float64) of what the GPU path computes.  Only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The product path (the HIP library and its Python binding) never
imports, links or calls anything in here, and nothing in here imports the
product package.

What it follows (Doi & Horii, "Cache Blocking Technique to Large Scale Quantum
Computing Simulation on Supercomputers", arXiv:2102.02957):

* state vector of 2^n complex amplitudes, qubit k <-> index bit k
  (Sec. II-A, Fig. "qb_array" and Fig. "u3_gate");
* the u3 gate of Eq. (1) and CNOT of Eq. (2), applied pair-wise on amplitudes
  whose indices differ in one bit (Sec. II-A);
* every other gate by its textbook matrix, applied per gate (no blocking, no
  fusion, no reordering): the cache-blocked method reaches exactly this product
  (Sec. IV-A: only commuting gates are reordered and the inserted chunk swaps
  are noiseless swaps);
* FP64 reductions (norm, overlap, fidelity, diagonal Z-string expectation);
* a plain adjoint gradient plus parameter-shift and finite differences;
* an executor for an exported blocked plan (Sec. IV-A, the transpiler's
  output: chunk swaps, begin/end of blocking sections);
* density-matrix evolution with noise channels, rho -> sum K rho K^dagger on
  the full 2^n x 2^n matrix (Sec. III-A: noisy simulation, density-matrix
  method), in ``oracle.density``.

Gates are plain tuples ``(kind, qubits, params, matrix, pidx)``; see
``oracle.gates`` for the kinds.
"""

from .gates import gate_matrix, u3_matrix, is_diagonal_kind, GATE_ARITY
from .statevector import (zero_state, basis_state, apply_gate, apply_circuit,
                          apply_matrix, apply_1q_pairwise, bind_params)
from .observables import (norm2, overlap, fidelity, max_abs_diff,
                          zstring_expval, ring_zz_terms, zz_diag_values)
from .adjoint import (adjoint_gradient, parameter_shift_gradient, parameter_shift_tail,
                      finite_difference_gradient, energy)
from .plan_exec import run_plan
from .closed_forms import qft_basis_amplitude, ghz_state
from . import density

__all__ = [
    "gate_matrix", "u3_matrix", "is_diagonal_kind", "GATE_ARITY",
    "zero_state", "basis_state", "apply_gate", "apply_circuit", "apply_matrix",
    "apply_1q_pairwise", "bind_params",
    "norm2", "overlap", "fidelity", "max_abs_diff", "zstring_expval",
    "ring_zz_terms", "zz_diag_values",
    "adjoint_gradient", "parameter_shift_gradient", "parameter_shift_tail", "finite_difference_gradient",
    "energy", "run_plan", "qft_basis_amplitude", "ghz_state", "density",
]
