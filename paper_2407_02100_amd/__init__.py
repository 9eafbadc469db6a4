"""MI355X (gfx950) vertex-patch multigrid smoother library: HIP kernels behind a C ABI.

``paper_2407_02100_amd.vps`` is the Python binding of ``libvps.so``; build the
library with ``python -m paper_2407_02100_amd.build``.
"""
from . import vps  # noqa: F401
from .vps import Context, VpsError  # noqa: F401
