"""Plain FP64 CPU oracle for the HOTRG coarse-graining step (arXiv 2306.00358).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or links
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP library (no kernels, headers, helpers or tables) and never receives a value
computed by it.

Modules
-------
tensors   initial site tensors (Ising, XY, Potts) built from Boltzmann weights
hotrg     the coarse-graining loop, step by step in the paper's order
exact     closed forms and brute force used to pin the oracle
          (Onsager's free energy, transfer matrices on tiny tori)

Every function states the passage of the paper it follows.  Pinned functions
are checked by ``tests/test_oracle_*.py`` against values fixed by the paper or
by mathematics other than the oracle itself.
"""

from . import tensors, hotrg, exact  # noqa: F401
