"""FP64 CPU oracle for TV/L2 reconstruction from random projections.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, the package's ``__graft_entry__.smoke()`` check and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code, table or helper with the GPU
path: the only common inputs are the seeded arrays drawn by
``paper_1001_1774_amd.synth``.

Every function follows the paper (Xiao and Yang, "A Fast Algorithm for Total
Variation Image Reconstruction from Random Projections") and cites the
section/equation it implements.  Parity status of each function is listed in
``tvcs_oracle.__doc__``.
"""
from .tvcs_oracle import *  # noqa: F401,F403
