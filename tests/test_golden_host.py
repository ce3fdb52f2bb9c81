"""Pins of the oracle's geometry to values the paper prints for its deployment
(tests/golden/lwa_sv_deployment.txt, Sec. 4.1-4.2; the paper gives no worked
numerical example of an image).

* the channelisation figures are mutually consistent and are the ones the
  synthetic inputs use;
* at a lambda/2 grid spacing the deployed 110 m aperture (plus its 3 m
  top-hat) spans about 41 cells at 55.25 MHz: it fits a 64-cell grid and not a
  32-cell one, which is the paper's "approximately 64^2 pixels" -- a wrong
  cell size (lambda instead of lambda/2, or metres per cell inverted) fails;
* at that spacing the image samples direction cosines over [-1, 1) (the
  paper's Nyquist, all-sky statement, Sec. 3.2): a plane wave from the
  horizon, l = -1, lands on the first pixel column.
"""
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "lwa_sv_deployment.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    return vals


G = _golden()


def _deployed_channels():
    n = int(G["n_channels_deployed"])
    return G["centre_hz"] + (np.arange(n) - (n - 1) / 2) * G["channel_width_hz"]


def test_channelisation_is_consistent_and_used_by_the_inputs():
    # a real-sampled band of fs / 2 cut into 4096 channels
    assert G["adc_sample_rate_hz"] / 2 / G["n_channels_total"] == G["channel_width_hz"]
    assert abs(1 / G["channel_width_hz"] - G["sample_time_s"]) < 1e-18
    assert G["n_channels_deployed"] * G["channel_width_hz"] == G["bandwidth_hz"]
    # 50 ms of 40 us samples: a whole number of samples per accumulated image
    n = G["accumulation_s"] / G["sample_time_s"]
    assert abs(n - 1250) < 1e-9
    assert synth.CHAN_BW_HZ == G["channel_width_hz"]
    assert synth.SAMPLE_S == G["sample_time_s"]


def _ellipse_edge(n=64):
    """Antennas on the boundary of the deployed ellipse (x east, y north)."""
    t = 2 * np.pi * np.arange(n) / n
    return np.stack([G["aperture_ew_m"] / 2 * np.cos(t), G["aperture_ns_m"] / 2 * np.sin(t)], 1)


def test_half_wavelength_grid_of_the_deployed_aperture_is_about_64_cells():
    f = _deployed_channels()
    xy = _ellipse_edge()
    du = G["cell_wavelengths"]
    N = int(G["grid_n"])
    X, Y = oracle.antenna_cells(xy, f, N, du)
    lam = oracle.C0 / f
    # the north-south extent in cells, tap footprint of the top-hat included
    span = (Y.max(axis=1) - Y.min(axis=1)) + G["tophat_m"] / (lam * du)
    assert np.all((span > N / 2) & (span < N)), span
    assert np.allclose(span, (G["aperture_ns_m"] + G["tophat_m"]) / (lam * du))
    # a 3 x 3 support covers the 3 m top-hat (about 1.1 cells) and stays on the
    # 64 grid; the same aperture does not fit a 32 grid
    assert np.all(G["tophat_m"] / (lam * du) <= 3)
    oracle.kernel_taps(X, Y, N, 3, 0.5)
    X32, Y32 = oracle.antenna_cells(xy, f, 32, du)
    with pytest.raises(oracle.OffGridError):
        oracle.kernel_taps(X32, Y32, 32, 3, 0.5)


def test_horizon_plane_wave_lands_on_the_first_column():
    """Antennas on whole cells at 55.25 MHz; a plane wave
    from l = -1, m = 0 has phase exp(-2 pi i u l) = (-1)^(cell offset) at each
    antenna (exact in int4).  The image, divided by the squared transform of
    the 3 x 3 Gaussian, peaks at pixel column 0, i.e. l = (0 - N/2) / (N du) = -1,
    with the value T |s|^2 A^2 expected there."""
    N, A, T, s = int(G["grid_n"]), 20, 3, 7.0
    du = G["cell_wavelengths"]
    f = np.array([G["centre_hz"]])
    cell_m = oracle.C0 / f[0] * du
    rng = np.random.default_rng(11)
    cells = set()
    while len(cells) < A:
        cells.add(tuple(rng.integers(-25, 26, size=2)))
    cxy = np.array(sorted(cells), dtype=float)
    cx = cxy[:, 0]
    xy = cxy * cell_m
    e = s * (-1.0) ** cx
    b = synth.pack_ci4(e, np.zeros(A))
    ef = np.broadcast_to(b[None, None, None, :], (T, 1, 1, A)).copy()
    g = np.ones((1, 1, A), np.complex64)
    img = oracle.image(xy, f, g, ef, N, 3, 0.5, du)[0, 0].real
    k = np.arange(N) - N // 2
    e2 = np.exp(-2.0)
    b1 = 1 + 2 * e2 * np.cos(2 * np.pi * k / N)
    B2 = np.outer(b1, b1) ** 2
    row, col = np.unravel_index(np.argmax(img / B2), img.shape)
    assert (row, col) == (N // 2, 0)
    assert (col - N / 2) / (N * du) == -1.0
    expect = T * s ** 2 * A ** 2 * B2[row, col]
    assert abs(img[row, col] - expect) / expect < 1e-12
