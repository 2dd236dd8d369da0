"""Seeded synthetic interferogram generator.

This module produces camera-like integer frames for the tests and the
benchmark.  It serves both the FP64 oracle and the HIP library as *input
data*; it contains none of the reconstruction arithmetic (no angular
spectrum, no single-FFT Fresnel transform, no STFT, no PCA).  Its forward
model builds the sensor-plane object wave by direct superposition of
paraxial point-source responses (a 1-D quadratic-phase kernel applied along
each axis as a matrix product), then adds a tilted plane reference and draws
Poisson photon counts.
"""

from .holograms import (  # noqa: F401
    HoloSpec,
    hologram_stack,
    config_c1,
    config_c2_block,
    config_c3,
    stream_block,
)
