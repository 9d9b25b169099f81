"""MI355X (gfx950) Hamilton-Jacobi reachability: Backward Reachable Tubes of
a 4D car by explicit Lax-Friedrichs time stepping on a grid (arXiv
2012.04011), as hand-written HIP kernels behind a C ABI (``include/hj.h``).

``paper_2012_04011_amd.hj`` is the ctypes binding (loads ``libhj.so`` on
first use); ``paper_2012_04011_amd.workloads`` holds the seeded synthetic
workloads.
"""

__all__ = ["hj", "workloads"]
