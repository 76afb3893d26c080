"""FP64 CPU oracle for the hyperuniform-field hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never imports, links or calls it, and it
shares no code, tables or helpers with that path.

What it computes follows Zhong & Mao, "Ultra-Efficient Reconstruction of
Anisotropic Hyperuniform Continuous Random Fields in 2D and 3D via Generalized
Spectral Filtering" (arXiv 2509.08675):

* white noise, then a forward FFT (Sec. II.B, the pipeline summary after Eq. (15));
* the amplitude filter A = sqrt(chi) of Eq. (8) with the superellipse norm of
  Eq. (12) inside the spectral density of Eq. (13);
* the inverse transform to a real field, Eq. (9);
* demean and rescale, Eq. (15);
* the sign map to a +-1 two-phase medium (Sec. II.B, last paragraphs);
* binned power spectra of the continuous and the +-1 field (the figure rows of
  Sec. III);
* the hyperuniformity diagnostics of Sec. II.A: the local variance over a spherical window
  (Eq. (1)) in its Fourier form, the small-k exponent of a binned spectrum and the class of
  Eqs. (6)-(7);
* a general level cut for a target volume fraction and the two-point probability function of
  the resulting two-phase map (Wiener-Khinchin, Eqs. (10)-(11)).

Where the paper is silent (noise generator, FFT sign, band centre, rotation,
Nyquist handling, binning) the readings are stated in each function.  Every
function here is pinned by ``tests/test_oracle_*.py`` against closed forms,
brute force or an independent implementation, except where a docstring says
"parity unpinned".
"""

from .philox import philox4x32_10, uniforms_from_words, box_muller, white_noise
from .spectral import (FilterParams, DegenerateFilter, wavenumbers_half, wavenumbers_full,
                       ln_chi_rel, amplitude_half, amplitude_sym, amplitude_full, k_star)
from .field import gen_field, threshold, pipeline
from .spectrum import bin_table, bin_power, power_spectrum, continuous_spectrum_fused
from .loss import (target_bins, spectrum_loss, spectrum_loss_grad, dlnH_half,
                   PARAM_NAMES)
from .diagnostics import form_factor, window_variance, small_k_exponent, hyperuniformity_class, CLASSES
from .twopoint import level_threshold, level_cut, s2_map, s2_brute

__all__ = [
    "philox4x32_10", "uniforms_from_words", "box_muller", "white_noise",
    "FilterParams", "DegenerateFilter", "wavenumbers_half", "wavenumbers_full",
    "ln_chi_rel", "amplitude_half", "amplitude_sym", "amplitude_full", "k_star",
    "gen_field", "threshold", "pipeline",
    "bin_table", "bin_power", "power_spectrum", "continuous_spectrum_fused",
    "target_bins", "spectrum_loss", "spectrum_loss_grad", "dlnH_half", "PARAM_NAMES",
    "form_factor", "window_variance", "small_k_exponent", "hyperuniformity_class", "CLASSES",
    "level_threshold", "level_cut", "s2_map", "s2_brute",
]
