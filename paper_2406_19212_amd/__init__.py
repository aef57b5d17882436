"""MI355X (gfx950) hot path of the JuliVQC variational-circuit method
(arXiv:2406.19212): gate and channel application on complex128 state vectors
and vectorised density matrices, Pauli-sum expectations and adjoint gradients,
as hand-written HIP kernels behind the C ABI in include/vqc.h.

``State``, ``Circuit`` and ``Batch`` wrap the C handles; torch supplies
device memory and the current stream.  Importing the package does not load
the library; the first handle does, and raises if it is not built.
"""
from .api import State, Circuit, Batch, fuse_gates, ops_params, stream_ptr  # noqa: F401
from . import workloads  # noqa: F401
