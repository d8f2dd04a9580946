"""MI355X (gfx950) fast damped Gauss-Newton (fLM) step for CANDECOMP/PARAFAC.

The computation lives in the HIP library libdgn.so (C ABI in include/dgn.h);
`paper_1205_2584_amd.dgn` is a thin ctypes binding that only marshals
arguments.  Importing this package loads nothing; the binding loads the
library on first use and raises if it has not been built.
"""

__all__ = ["dgn", "build"]
