"""MI355X (gfx950) multi-layer PET Monte Carlo: HIP kernels behind a C ABI.

The library ``libgpet.so`` (sources in ``csrc/``, API in ``include/gpet.h``)
transports back-to-back 511 keV photon pairs through a voxelized phantom and a
panel -> module -> layer -> crystal detector and digitizes the hits.
:class:`paper_2603_07327_amd.gpet.Context` is the Python binding.
"""
from .gpet import Context, GpetError, load_library  # noqa: F401
