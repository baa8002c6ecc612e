"""FP64 CPU oracle of the Triad-ATRG method (arXiv:2412.14104).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the cpu_baseline
leg of bench.py, never by the product library.  It shares no code with the HIP path.
"""
import numpy as _np

# Large temporaries are touched once; asking the kernel for transparent huge pages on them
# makes first-touch page faults compact memory synchronously, which costs far more than it
# saves here.  This changes speed only, never values.
try:
    _np._core.multiarray._set_madvise_hugepage(False)
except AttributeError:  # older numpy layout
    try:
        _np.core.multiarray._set_madvise_hugepage(False)
    except AttributeError:
        pass
