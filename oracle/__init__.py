"""FP64 CPU oracle for the state-vector gate sweep of Tabakin & Julia-Diaz, QCMPI.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
helpers with the HIP library; the two meet only in the seeded input generator
(``paper_0902_0699_amd/workload.py``), which holds none of the method's
arithmetic.

Every function is plain NumPy ``complex128`` arithmetic that follows the
paper's definitions literally (one gate at a time, no fusion, no deferred
scaling).  Each function names the passage it follows.  All functions are
pinned by ``tests/test_oracle_pins.py`` against worked examples, closed forms,
library routines and brute force; none is "parity unpinned".
"""

from .qcmpi import *  # noqa: F401,F403
