"""FP64 CPU oracle for the IPOP-CMA-ES generation path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python binding
may import, call or link this package; only the test suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
path: it has its own Philox generator, its own parameter formulas and its own
update arithmetic, written plainly in NumPy float64 so that it can be checked
against the paper by eye.

Parity pins (what each function is checked against) are listed in the header
of ``cmaes_oracle.py``.
"""

from .cmaes_oracle import *  # noqa: F401,F403
