"""FP64 reductions on state vectors (TEST INFRASTRUCTURE ONLY).

All sums use NumPy's pairwise summation in float64 / complex128.
"""

import numpy as np


def norm2(psi):
    """<psi|psi> = sum_x |a_x|^2."""
    a = np.asarray(psi, dtype=np.complex128)
    return float(np.sum(a.real * a.real + a.imag * a.imag))


def overlap(a, b):
    """<a|b> = sum_x conj(a_x) b_x."""
    return complex(np.vdot(np.asarray(a, dtype=np.complex128), np.asarray(b, dtype=np.complex128)))


def fidelity(a, b):
    """Normalised fidelity F = |<a|b>|^2 / (<a|a><b|b>)."""
    ov = overlap(a, b)
    return (ov.real ** 2 + ov.imag ** 2) / (norm2(a) * norm2(b))


def max_abs_diff(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.complex128) - np.asarray(b, dtype=np.complex128))))


def ring_zz_terms(n):
    """H = sum_i Z_i Z_{(i+1) mod n} as (coefficient, Z-mask) terms."""
    if n == 1:
        return [(1.0, 0)]
    if n == 2:
        # Z0Z1 appears twice in the periodic ring of two qubits.
        return [(2.0, 0b11)]
    return [(1.0, (1 << i) | (1 << ((i + 1) % n))) for i in range(n)]


def zz_diag_values(n, terms):
    """h(x) = sum_t c_t * prod_{i in mask_t} z_i(x), z_i = 1 - 2 bit_i(x)."""
    x = np.arange(1 << n, dtype=np.int64)
    h = np.zeros(1 << n, dtype=np.float64)
    for coeff, mask in terms:
        sign = np.ones(1 << n, dtype=np.float64)
        for i in range(n):
            if (mask >> i) & 1:
                sign *= 1.0 - 2.0 * ((x >> i) & 1)
        h += coeff * sign
    return h


def zstring_expval(psi, n, terms):
    """E = sum_x |a_x|^2 h(x) for a diagonal observable given as Z-strings."""
    a = np.asarray(psi, dtype=np.complex128)
    p = a.real * a.real + a.imag * a.imag
    return float(np.sum(p * zz_diag_values(n, terms)))
