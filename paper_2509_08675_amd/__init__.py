"""MI355X-native generator of anisotropic hyperuniform continuous random fields.

The hot path of Zhong & Mao, arXiv 2509.08675 (single-shot generalized-superellipse spectral
filtering): seeded white noise, forward FFT, superellipse filter, inverse FFT, normalisation,
sign threshold and binned power spectra, as HIP kernels for gfx950 behind the C-ABI of
include/hufield.h.  ``paper_2509_08675_amd.hufield`` is the Python binding (it needs the built
libhufield.so and a GPU for any compute call); ``workloads`` names the synthetic workloads.
"""

from . import workloads

__all__ = ["workloads"]
