"""FP64 CPU oracle for the MOFF direct imager.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library.  See oracle/moff.py for what each function follows.
"""
from .moff import (C0, OffGridError, unpack_ci4, antenna_cells, kernel_taps,  # noqa: F401
                   grid_efield, transform, direct_dft, products, n_products, image,
                   image_from, aperture_response, visibilities, image_fx, grad_gains,
                   l2_loss, l2_loss_grad_image, fd_grad, fd_directional, model_image,
                   rel_errors, auto_visibilities, autocorrelation_image, image_without_autos,
                   image_without_autos_from, grad_autos, grad_gains_without_autos,
                   decimate_transpose, pseudo_stokes, kernel_taper, taper_corrected)
