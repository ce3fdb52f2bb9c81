"""Plant plausible mistakes in the oracle (on the CPU only) and check that the
pins catch each one: the pins must not pass for a wrong oracle."""
import numpy as np
import pytest

import oracle
from oracle import moff
import tests.test_golden_host as golden
import tests.test_oracle_pins as pins

_transform = moff.transform
_products = moff.products
_kernel_taps = moff.kernel_taps
_grad = moff.grad_gains
_auto_vis = moff.auto_visibilities
_front = moff.decimate_transpose
_stokes = moff.pseudo_stokes
_taper = moff.kernel_taper
_cells = moff.antenna_cells
_model = moff.model_image
_rel_errors = moff.rel_errors


def _wrong_sign(a):
    return np.fft.fft2(a, axes=(-2, -1))


def _transposed(a):
    return np.swapaxes(_transform(a), -1, -2)


def _unscaled(a):
    return np.fft.ifft2(a, axes=(-2, -1))


def _xy_without_conj(F):
    out = _products(F)
    if F.shape[1] == 2:
        out[:, 1] = F[:, 0] * F[:, 1]
        out[:, 2] = np.conj(out[:, 1])
    return out


def _sigma_not_squared(X, Y, grid_n, support=3, sigma_cells=0.5, kernels=None):
    ii, jj, w = _kernel_taps(X, Y, grid_n, support, sigma_cells)
    d2 = (ii - X[..., None]) ** 2 + (jj - Y[..., None]) ** 2
    return ii, jj, np.exp(-d2 / (2.0 * sigma_cells))


def _taps_rounded_down(X, Y, grid_n, support=3, sigma_cells=0.5, kernels=None):
    """Nearest cell taken as floor(X) instead of floor(X + 1/2)."""
    ii, jj, _ = _kernel_taps(X - 0.5, Y - 0.5, grid_n, support, sigma_cells)
    d2 = (ii - X[..., None]) ** 2 + (jj - Y[..., None]) ** 2
    return ii, jj, np.exp(-d2 / (2.0 * sigma_cells ** 2))


def _grad_half(*a, **k):
    return 0.5 * _grad(*a, **k)


def _autos_not_squared(xy_m, freq_hz, gains, efield, grid_n, kernel_support=3,
                       kernel_sigma_cells=0.5, cell_wavelengths=0.5, kernels=None):
    b = moff.aperture_response(xy_m, freq_hz, grid_n, kernel_support, kernel_sigma_cells,
                               cell_wavelengths, kernels)
    out = np.einsum("cka,cayx->ckyx", moff.auto_visibilities(gains, efield), np.abs(b))
    return np.fft.fftshift(out, axes=(-2, -1))


def _grad_autos_variant(conj_sxy=True, two=2.0):
    """grad_autos with one planted slip (the cross term's conjugate, the factor 2)."""
    def fn(xy_m, freq_hz, gains, efield, grid_n, grad_image, kernel_support=3,
           kernel_sigma_cells=0.5, cell_wavelengths=0.5, kernels=None):
        B = np.abs(moff.aperture_response(xy_m, freq_hz, grid_n, kernel_support,
                                          kernel_sigma_cells, cell_wavelengths, kernels)) ** 2
        gam = np.fft.ifftshift(np.asarray(grad_image).astype(complex), axes=(-2, -1))
        e = moff.unpack_ci4(efield)
        g = np.asarray(gains).astype(complex)
        out = np.zeros(g.shape, complex)
        out[:, 0] = two * np.einsum("cyx,cayx->ca", gam[:, 0].real, B) \
            * np.sum(np.abs(e[:, :, 0]) ** 2, axis=0) * g[:, 0]
        if g.shape[1] == 2:
            s_xy = np.sum(e[:, :, 0] * np.conj(e[:, :, 1]), axis=0)
            h = np.einsum("cyx,cayx->ca", gam[:, 1] + np.conj(gam[:, 2]), B)
            out[:, 0] += h * (np.conj(s_xy) if conj_sxy else s_xy) * g[:, 1]
            out[:, 1] = two * np.einsum("cyx,cayx->ca", gam[:, 3].real, B) \
                * np.sum(np.abs(e[:, :, 1]) ** 2, axis=0) * g[:, 1] + np.conj(h) * s_xy * g[:, 0]
        return out
    return fn


def _front_pol_antenna_swapped(raw, n_chan, c0=0, c_step=1):
    out = _front(raw, n_chan, c0, c_step)
    return np.ascontiguousarray(out.reshape(out.shape[0], out.shape[1], out.shape[3], out.shape[2])
                                .transpose(0, 1, 3, 2)) if out.shape[2] != out.shape[3] else out


def _front_step_ignored(raw, n_chan, c0=0, c_step=1):
    return _front(raw, n_chan, c0, 1)


def _kernels_conjugated(X, Y, grid_n, support=3, sigma_cells=0.5, kernels=None):
    ii, jj, w = _kernel_taps(X, Y, grid_n, support, sigma_cells, kernels)
    return ii, jj, np.conj(w)


def _grad_kernel_unconjugated(xy_m, freq_hz, gains, efield, grid_n, grad_image, kernel_support=3,
                              kernel_sigma_cells=0.5, cell_wavelengths=0.5, chunk=128,
                              kernels=None):
    if kernels is None:
        return _grad(xy_m, freq_hz, gains, efield, grid_n, grad_image, kernel_support,
                     kernel_sigma_cells, cell_wavelengths, chunk, kernels)
    X, Y = moff.antenna_cells(xy_m, freq_hz, grid_n, cell_wavelengths)
    ii, jj, w = _kernel_taps(X, Y, grid_n, kernel_support, kernel_sigma_cells, kernels)
    # recompute with the kernel left unconjugated in the degridding
    e_all = moff.unpack_ci4(np.asarray(efield))
    gg = np.asarray(gains).astype(complex)
    Gam = np.fft.ifftshift(np.asarray(grad_image).astype(complex), axes=(-2, -1))
    out = np.zeros(gg.shape, complex)
    for c in range(gg.shape[0]):
        e = e_all[:, c]
        F = moff.transform(moff.grid_efield(gg[c][None] * e, ii[c], jj[c], w[c], grid_n))
        if gg.shape[1] == 1:
            G = (Gam[c, 0].real * F[:, 0])[:, None]
        else:
            h = 0.5 * (Gam[c, 1] + np.conj(Gam[c, 2]))
            G = np.stack([Gam[c, 0].real * F[:, 0] + h * F[:, 1],
                          Gam[c, 3].real * F[:, 1] + np.conj(h) * F[:, 0]], axis=1)
        H = np.fft.fft2(G, axes=(-2, -1))
        out[c] = np.einsum("ak,tpak,tpa->pa", w[c], H[:, :, jj[c], ii[c]], np.conj(e))
    return 2.0 * out


def _cells_of_one_wavelength(xy_m, freq_hz, grid_n, cell_wavelengths=0.5):
    """Grid cells one wavelength wide whatever the spacing asked for."""
    return _cells(xy_m, freq_hz, grid_n, 1.0)


def _stokes_v_flipped(img):
    out = _stokes(img)
    if out.shape[1] == 4:
        out[:, 3] *= -1
    return out


def _taper_not_squared(*a, **k):
    return np.sqrt(_taper(*a, **k))


def _auto_vis_swapped(gains, efield):
    v = _auto_vis(gains, efield)
    if v.shape[1] == 4:
        v = v[:, [0, 2, 1, 3]]
    return v


def _model_sources_mirrored(xy_m, freq_hz, grid_n, n_time, src_lm, src_power, noise_sigma, **k):
    """Source phase exp(+2 pi i (u l + v m)): every model source lands at -(l, m)."""
    return _model(xy_m, freq_hz, grid_n, n_time, -np.asarray(src_lm), src_power, noise_sigma, **k)


def _model_noise_without_two(xy_m, freq_hz, grid_n, n_time, src_lm, src_power, noise_sigma, **k):
    """Noise visibility sigma^2 Id instead of 2 sigma^2 Id (one component only)."""
    return _model(xy_m, freq_hz, grid_n, n_time, src_lm, src_power, noise_sigma / np.sqrt(2), **k)


def _model_per_sample(xy_m, freq_hz, grid_n, n_time, src_lm, src_power, noise_sigma, **k):
    """The model of one sample, not of the integration."""
    return _model(xy_m, freq_hz, grid_n, 1, src_lm, src_power, noise_sigma, **k)


def _rel_errors_xy_own_norm(img, ref):
    """XY and YX measured against their own norm."""
    out = _rel_errors(img, ref)
    if img.shape[1] == 4:
        d = np.linalg.norm((img - ref).reshape(img.shape[0], 4, -1), axis=-1)
        r = np.linalg.norm(ref.reshape(ref.shape[0], 4, -1), axis=-1)
        out[:, 1:3] = d[:, 1:3] / np.maximum(r[:, 1:3], 1e-300)
    return out


def _rel_errors_xy_by_xx(img, ref):
    """XY and YX scaled by ||XX|| alone."""
    out = _rel_errors(img, ref)
    if img.shape[1] == 4:
        d = np.linalg.norm((img - ref).reshape(img.shape[0], 4, -1), axis=-1)
        r = np.linalg.norm(ref.reshape(ref.shape[0], 4, -1), axis=-1)
        out[:, 1:3] = d[:, 1:3] / r[:, :1]
    return out


MUTATIONS = {
    "transform with the -i sign": ("transform", _wrong_sign,
                                   [pins.test_p1_transform_sign_single_cell]),
    "rows and columns swapped": ("transform", _transposed,
                                 [lambda: pins.test_p2_plane_wave_lands_on_its_pixel(8, 0)]),
    "transform normalised by 1/n_g": ("transform", _unscaled, [pins.test_p3_parseval]),
    "XY without the conjugate": ("products", _xy_without_conj,
                                 [lambda: pins.test_p5_fx_form_equals_moff(21, 32, 16, 2, 2, 6)]),
    "kernel width not squared": ("kernel_taps", _sigma_not_squared,
                                 [pins.test_kernel_weights_closed_form]),
    "taps centred half a cell off": ("kernel_taps", _taps_rounded_down,
                                     [pins.test_p2_zenith_closed_form_off_cell]),
    "gradient without the factor 2": ("grad_gains", _grad_half,
                                      [lambda: pins.test_p10_gradient_matches_finite_differences(1)]),
    "autocorrelations with |b| not squared": ("autocorrelation_image", _autos_not_squared,
                                              [pins.test_p13_autos_removed_equals_fx_form_without_diagonal]),
    "XY and YX autocorrelations swapped": ("auto_visibilities", _auto_vis_swapped,
                                           [pins.test_p13_autos_removed_equals_fx_form_without_diagonal]),
    "autocorrelation gradient with s_XY not conjugated": (
        "grad_autos", _grad_autos_variant(conj_sxy=False),
        [pins.test_p14_gradient_without_autos_cross_products_only,
         lambda: pins.test_p14_gradient_without_autos_matches_finite_differences(2)]),
    "front end reading [A, P] as [P, A]": (
        "decimate_transpose", _front_pol_antenna_swapped,
        [lambda: pins.test_p15_decimate_transpose_by_loops(0, 1, 5, 2)]),
    "front end ignoring the channel step": (
        "decimate_transpose", _front_step_ignored,
        [lambda: pins.test_p15_decimate_transpose_by_loops(1, 2, 3, 1)]),
    "user kernels conjugated in the gridding": (
        "kernel_taps", _kernels_conjugated, [pins.test_p16_kernel_phase_moves_into_the_gain]),
    "gradient degridding with the kernel unconjugated": (
        "grad_gains", _grad_kernel_unconjugated,
        [lambda: pins.test_p16_gradient_with_complex_kernels_matches_finite_differences(2)]),
    "Stokes V with the opposite sign": (
        "pseudo_stokes", _stokes_v_flipped,
        [lambda: pins.test_p17_pseudo_stokes_of_pure_polarisation_states(4, 4j, 0, 0, -1)]),
    "kernel taper not squared": (
        "kernel_taper", _taper_not_squared,
        [pins.test_p17_taper_correction_is_exact_for_identical_kernels]),
    "grid cells a whole wavelength wide": (
        "antenna_cells", _cells_of_one_wavelength,
        [golden.test_half_wavelength_grid_of_the_deployed_aperture_is_about_64_cells]),
    "autocorrelation gradient without the factor 2": (
        "grad_autos", _grad_autos_variant(two=1.0),
        [lambda: pins.test_p14_gradient_without_autos_matches_finite_differences(1),
         pins.test_p14_homogeneity_without_autos]),
    "model sources at the mirrored direction": (
        "model_image", _model_sources_mirrored,
        [lambda: pins.test_p18_model_image_whole_cell_closed_form(2)]),
    "model noise term without the factor 2": (
        "model_image", _model_noise_without_two,
        [lambda: pins.test_p18_model_image_whole_cell_closed_form(1),
         pins.test_p18_model_image_zenith_off_cell]),
    "model of one sample instead of the integration": (
        "model_image", _model_per_sample, [pins.test_p18_model_image_zenith_off_cell]),
    "error metric: XY against its own norm": (
        "rel_errors", _rel_errors_xy_own_norm, [pins.test_p19_error_metric_hand_values]),
    "error metric: XY scaled by ||XX|| alone": (
        "rel_errors", _rel_errors_xy_by_xx, [pins.test_p19_error_metric_hand_values]),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_pins_catch_planted_mistake(name, monkeypatch):
    attr, fn, checks = MUTATIONS[name]
    monkeypatch.setattr(moff, attr, fn)
    monkeypatch.setattr(oracle, attr, fn)
    for check in checks:
        with pytest.raises(AssertionError):
            check()
