"""MI355X (gfx950) implementation of the implicit APIC MPM hot path with spatially varying
surface energy (Chen et al., arXiv 2101.12408).

The computation lives in libmpm.so (HIP kernels + C ABI, include/mpm.h); this package is
the Python binding.  Build the library with `python -m paper_2101_12408_amd.build`.
"""
from ._lib import LIB_PATH, load  # noqa: F401
from .api import (MpmError, Scene, make_params, mpm_energy_grad, mpm_g2p, mpm_heat_apply,  # noqa: F401
                  mpm_hessvec, mpm_p2g, mpm_step, sample_surface, tiled_index)
