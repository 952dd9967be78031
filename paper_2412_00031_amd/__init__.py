"""MI355X-native hot path of adjoint-state traveltime tomography (TomoATT,
arXiv 2412.00031): batched fast-sweeping Eikonal solves, discrete adjoint
solves and sensitivity kernels in hand-written HIP kernels (libtt.so).

Importing the package loads nothing; ``api`` loads libtt.so on first use and
raises if it has not been built.
"""

__all__ = ["api", "workloads"]
