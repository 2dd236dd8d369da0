"""FP64 CPU oracle for the hologram-rendering hot path.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the HIP library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path (``paper_2508_03911_amd``) never does, and this package imports
nothing from the product path.  The two share no code: every transform here is
written from its mathematical definition with numpy in float64/complex128.

What it follows (paper: "Holovibes: Real-time Ultrahigh-Speed Digital Hologram
Rendering and Short-Time Analysis", arXiv 2508.03911):

* Sec. III-B.1 (Space and time transformations): camera integers converted to
  complex, a per-frame spatial transform (angular-spectrum propagation or a
  Fresnel transform, both named in the Abstract and Sec. II-B.3), a temporal
  transform over a user-sized window of consecutive reconstructed frames
  (short-time Fourier transform, or PCA through covariance,
  eigendecomposition and projection onto a sub-basis), then a per-pixel
  statistical moment over a range of temporal indices.
* Sec. VI-B (benchmarks): the two pipelines "angular spectrum + STFT" and
  "Fresnel + PCA", window equal to stride.

The paper gives these operations in words only.  The formulas below are
textbook readings (sign of z, normalisation, band-to-bin mapping, PCA
conventions); each function's docstring states the reading it implements.
Modules:

* ``optics``    -- unpack, angular spectrum, single-FFT Fresnel transform.
* ``temporal``  -- STFT windows, band-to-bin mapping, Doppler moments.
* ``pca``       -- covariance, ordered eigendecomposition, projection energy.
* ``ssa``       -- the SSA + FFT path: components c1..c2 of each window, then the STFT.
* ``pipeline``  -- the end-to-end compositions used by the tests.
* ``autofocus`` -- the z-scan sharpness reference and the FP64 CNN.
* ``post``      -- magnitude and argument images, post-processing chain.
* ``holo``      -- the .holo file layout.
"""

from . import optics, temporal, pca, ssa, pipeline  # noqa: F401
