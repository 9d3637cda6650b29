"""Closed-form amplitudes usable at any qubit count (TEST INFRASTRUCTURE ONLY).

They let a 33- or 34-qubit result be checked one sampled amplitude at a time,
without holding the state on the host.
"""

import cmath
import math

import numpy as np


def qft_basis_amplitude(n, x, y):
    """<y| QFT |x> = exp(2 pi i x y / 2^n) / sqrt(2^n).

    The QFT named in Sec. V-A as a workload; the product x*y is reduced
    modulo 2^n in exact integer arithmetic so the phase keeps full precision
    at large n.
    """
    big = 1 << n
    r = (int(x) * int(y)) % big
    return cmath.exp(2j * math.pi * (r / big)) / math.sqrt(big)


def qft_basis_amplitudes(n, x, ys):
    return np.array([qft_basis_amplitude(n, x, int(y)) for y in ys], dtype=np.complex128)


def ghz_state(n):
    """(|0...0> + |1...1>) / sqrt(2)."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = psi[-1] = 1.0 / math.sqrt(2.0)
    return psi
