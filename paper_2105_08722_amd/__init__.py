"""MI355X (gfx950) hot path of the discrete isotropic N-point correlation function
estimator (Philcox et al. 2021): HIP kernels behind a C ABI (include/encore.h),
with a thin ctypes binding (paper_2105_08722_amd.encore)."""
from . import encore  # noqa: F401
