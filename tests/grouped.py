"""Expected amplitudes of a product-structured circuit from the oracle.

For a circuit whose gates stay inside disjoint qubit groups, the final state is
the tensor product of the groups' states.  Each group's circuit is run by the
oracle on its own small register (group qubit j -> local qubit j); an amplitude
of the full state at index x is the product over groups of the group state's
amplitude at the bits of x on that group's qubits.
"""

import numpy as np

import oracle


def group_states(gates, groups, psi_groups=None):
    """Oracle state of every group (list of 2^len(g) complex128 arrays)."""
    out = []
    for gi, grp in enumerate(groups):
        local = {q: j for j, q in enumerate(grp)}
        sub = []
        for g in gates:
            if all(q in local for q in g[1]):
                sub.append((g[0], tuple(local[q] for q in g[1]), g[2], g[3],
                            g[4] if len(g) > 4 else -1))
            else:
                assert not any(q in local for q in g[1]), "gate straddles groups"
        psi0 = None if psi_groups is None else psi_groups[gi]
        out.append(oracle.apply_circuit(len(grp), sub, psi0))
    return out


def product_amplitudes(states, groups, xs):
    """Amplitudes of the product state at the indices xs (uint64 array)."""
    xs = np.asarray(xs, dtype=np.uint64)
    amp = np.ones(len(xs), dtype=np.complex128)
    for st, grp in zip(states, groups):
        sub = np.zeros(len(xs), dtype=np.int64)
        for j, q in enumerate(grp):
            sub |= (((xs >> np.uint64(q)) & np.uint64(1)).astype(np.int64)) << j
        amp *= st[sub]
    return amp
