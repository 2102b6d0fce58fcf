"""MI355X-native relativistic space-charge FMM (arXiv 2302.07567).

The hot path (tree, interaction lists, P2M/M2M, P2P, M2L, L2L/L2P) runs in the
HIP library built from ``csrc/`` for gfx950 and is reached through the C-ABI
of ``include/relfmm.h``; ``binding`` holds the ctypes marshalling.  Importing
this package loads nothing; the library is loaded on first use and its
absence is an error.
"""
from .binding import Params, Plan, compute_fields, fields  # noqa: F401
