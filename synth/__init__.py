"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package produces *data only*: latent images, point-spread functions, blurred and
noisy observations, and the workload descriptions of the benchmark configurations.  It
contains none of the Richardson-Lucy arithmetic (no ratio, no adjoint correlation, no
update).  The one convolution it performs -- blurring the latent image to make the
observation f = g*h + n of the blur model (Section 1, eq. 1) -- is delegated to
``scipy.ndimage.convolve`` so that neither the oracle nor the HIP path is involved in
making their own inputs.
"""
from .psf import (box_h, box_v, box_rect, disc, disc_support_size, oblique_line,
                  dense_random, delta, normalise_to_f32)
from .images import latent_image, blur_reflect, observe
from .configs import CONFIGS, make_job, job_for_config

__all__ = [
    "box_h", "box_v", "box_rect", "disc", "disc_support_size", "oblique_line",
    "dense_random", "delta", "normalise_to_f32", "latent_image", "blur_reflect",
    "observe", "CONFIGS", "make_job", "job_for_config",
]
