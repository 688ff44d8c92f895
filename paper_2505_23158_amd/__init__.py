"""MI355X (gfx950) per-frame renderer for level-of-detail Gaussian splatting
(LODGE, arXiv 2505.23158): HIP kernels behind the C ABI of include/lodge.h,
with a ctypes binding (``lodge``), a differentiable wrapper (``autograd``)
and a continuous-batching render server (``serve``)."""
from . import lodge  # noqa: F401
