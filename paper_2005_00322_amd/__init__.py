"""MI355X-native hot path of the sine/cosine-basis PSTD method (arXiv:2005.00322).

The computation runs in the HIP kernels of ``libpstd.so`` (built from ``csrc/`` for gfx950); this
package only marshals arguments across its C ABI (``include/pstd.h``).  PyTorch supplies device memory
and the current stream.  There is no CPU fallback: every call raises if the library is missing.
"""
from .pstd import (DIRICHLET, DIRICHLET_HALF, GRAD_NODES, GRAD_STAG, NEUMANN, NEUMANN_HALF, NODES_TO_STAG,
                   PERIODIC, STAG_TO_NODES, Batch,
                   Plan, PstdError, State, axis_operator, combine_R,
                   combine_fields, face_weights, lib_path, load_library, solve_faces, solve_faces_2d)

__all__ = ["Plan", "Batch", "State", "PstdError", "combine_R", "combine_fields", "face_weights", "solve_faces", "solve_faces_2d",
           "axis_operator", "NEUMANN", "DIRICHLET", "PERIODIC", "NEUMANN_HALF", "DIRICHLET_HALF", "GRAD_NODES", "GRAD_STAG", "NODES_TO_STAG",
           "STAG_TO_NODES", "load_library", "lib_path"]
