"""qsv: cache-blocked state-vector gate application on one AMD MI355X (gfx950).

The compute path is the HIP library ``libqsv.so`` built from ``csrc/`` and
reached through its C ABI (``include/qsv.h``); ``binding`` marshals arguments
to it.  ``workloads`` holds the seeded synthetic circuits.
"""

__all__ = ["binding", "workloads"]
