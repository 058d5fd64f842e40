"""MI355X (gfx950) composite-grid AMR multigrid Poisson path for electrostatic
PIC after arXiv:1812.03689: HIP kernels behind the C ABI in include/amrmg.h,
with a ctypes binding (``paper_1812_03689_amd.amrmg``)."""
from . import workloads  # noqa: F401
