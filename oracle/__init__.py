"""FP64 CPU oracle for template-matching orientation mapping.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import, call or execute anything in this
package. The GPU library never routes through it, and it imports nothing from
the GPU library (a test checks both directions).

What it computes is the paper's indexation procedure (Section 2.2) written
out plainly, in float64, one function per step:

* ``intensity_transform64`` - gamma correction and constant subtraction of
  the experimental pattern (Section 2.2, discussion of the limitations of Q;
  Section 4.3 for the unit-intensity / subtract-constant workflow);
* ``polar64`` - polar resampling of a pattern about the direct-beam centre
  (Section 2.2, Fig. 2 c);
* ``template_pixels64`` - template spots rounded to integer polar pixels,
  mirrored templates by reflection across y = 0 (Section 2.2, Fig. 2 d);
* ``scores64`` / ``match_exact64`` - the correlation index Q of Eq. (1) at
  every in-plane shift with wraparound, and its maximum per template
  (Section 2.2, Fig. 2 e);
* ``topn64`` - sort and keep the N best templates (Section 2.2, end);
* ``refine_angle64`` - sub-bin in-plane angle by a parabola through the
  scores at the best shift and its neighbours (Section 5, discussion);
* ``prefilter64`` - azimuthally integrated pre-filter of the library
  (Section 2.2, Fig. 3);
* ``fft_match64`` - the same in-plane search through Fourier transforms
  along the azimuth (Section 2.2, computational cost);
* ``matrix_mask64`` - the mask of the dominant phase's reflections for
  two-stage indexing (Section 4.3, custom indexation procedures);
* ``match_orientation64`` / ``ipf_deviation64`` - Bunge Euler angles of a
  match (Section 2.1, Section 2.2 for mirrors) and the angular deviation
  between two orientation maps, Eq. (2) (Section 4.1);
* ``simulate_library64`` - kinematical template library: reciprocal grid,
  rotation, excitation error, shape and structure factors, projection
  (Section 2.1);
* ``preprocess64`` - direct-beam centring, difference-of-Gaussians
  background removal, Gaussian blur and thresholding (Section 4.1).

Readings where the paper is silent are stated in each function.
"""
from .polar import (polar_coords64, bilinear64, intensity_transform64,
                    polar64, norm64, profile64)
from .library import template_pixels64, OracleLibrary
from .match import (scores64, match_exact64, topn64, index_pattern64, index_batch64,
                    refine_angle64)
from .fft import template_images64, fft_numerators64, fft_match64
from .prefilter import radial_profiles64, prefilter64, index_pattern_prefiltered64
from .mask import mean_pattern64, binary_erode64, binary_dilate64, matrix_mask64
from .simulate import (reciprocal_grid64, structure_factor_sq64, reflections64,
                       excitation_error64, shape_factor64, simulate_template64,
                       simulate_library64)
from .preprocess import (gaussian_weights64, convolve_axis64, gaussian64, beam_centre64,
                         shift_image64, preprocess64)
from .orient import (bunge_matrix64, euler_from_matrix64, match_orientation64,
                     symmetry_operators64, in_sector64, sector_direction64,
                     ipf_deviation64)

__all__ = [
    "polar_coords64", "bilinear64", "intensity_transform64", "polar64", "norm64",
    "profile64", "template_pixels64", "OracleLibrary", "scores64", "match_exact64",
    "topn64", "index_pattern64", "index_batch64", "radial_profiles64", "prefilter64",
    "index_pattern_prefiltered64", "template_images64", "fft_numerators64", "fft_match64",
    "mean_pattern64", "binary_erode64", "binary_dilate64", "matrix_mask64", "refine_angle64",
    "bunge_matrix64", "euler_from_matrix64", "match_orientation64", "symmetry_operators64",
    "sector_direction64", "ipf_deviation64", "in_sector64", "reciprocal_grid64",
    "structure_factor_sq64", "reflections64", "excitation_error64", "shape_factor64",
    "simulate_template64", "simulate_library64", "gaussian_weights64", "convolve_axis64",
    "gaussian64", "beam_centre64", "shift_image64", "preprocess64",
]
