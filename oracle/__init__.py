"""CPU oracle for the MPMC hard-disk sampler — TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does.
"""
from .orc import OracleBox, philox, hist_edges, pressure_fit, acf, tau_fit, tau_int  # noqa: F401
