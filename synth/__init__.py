"""Seeded synthetic LWA-like inputs for the MOFF direct imager.

This module only *makes inputs*: antenna layouts, channel frequencies, complex
gains and channelised 4+4-bit E-field bytes.  It holds none of the imaging
arithmetic (no gridding kernel, no transform, no products).  Both the FP64
oracle and the GPU library are fed from here, so neither depends on the other.

Shapes and statistics follow the paper's instrument (Kent et al. 2019, §4.1:
256 dual-polarisation dipoles in a ~100 m aperture, 25 kHz channels sampled
every 40 us, 4+4-bit complex samples; §3.2: data ordered
[Time, Channel, Polarisation, Antenna] after transposition).

E-field model (readings, stated once here):
  * a point source k at direction (l_k, m_k) reaches antenna a with the
    geometric phase exp(-2 pi i (u_a l_k + v_a m_k)), u_a = x_a / lambda_c;
    under the +i spatial transform of §2.1 Eq. (5) it then appears at +(l_k, m_k);
  * its time series is a unit-modulus random phasor s(t) = exp(i phi_t), the
    same at every antenna; X and Y are independent for unpolarised sources;
  * receiver noise is complex Gaussian, sigma per component;
  * samples are quantised with round-half-to-even, clipped to [-8, 7] and
    packed as one byte: high nibble = real part, low nibble = imaginary part,
    both two's complement.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

C0 = 299_792_458.0          # speed of light, m/s
CHAN_BW_HZ = 25_000.0       # LWA channel width (§4.1)
SAMPLE_S = 40e-6            # one time sample per channel (§4.1)


@dataclasses.dataclass
class Inputs:
    """One imaging problem: geometry + gains + packed E-field bytes."""
    grid_n: int
    n_chan: int
    n_pol: int
    n_ant: int
    kernel_support: int
    kernel_sigma_cells: float
    cell_wavelengths: float
    xy_m: np.ndarray            # float64 [A, 2]  (east, north) metres
    freq_hz: np.ndarray         # float64 [C]
    gains: np.ndarray           # complex64 [C, P, A]
    efield: np.ndarray          # uint8 [T, C, P, A]
    sources: Optional[dict] = None
    name: str = ""
    kernels: Optional[np.ndarray] = None   # complex64 [C, A, K, K] user kernels, or None

    @property
    def n_time(self) -> int:
        return int(self.efield.shape[0])

    def config_dict(self) -> dict:
        return dict(grid_n=self.grid_n, n_chan=self.n_chan, n_pol=self.n_pol,
                    n_ant=self.n_ant, kernel_support=self.kernel_support,
                    kernel_sigma_cells=self.kernel_sigma_cells,
                    cell_wavelengths=self.cell_wavelengths)


# ---------------------------------------------------------------- encoding
def pack_ci4(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Quantise real/imag parts and pack them into 4+4-bit bytes.

    round-half-to-even, clip to [-8, 7]; high nibble = re, low nibble = im.
    """
    qr = np.clip(np.rint(re), -8, 7).astype(np.int16)
    qi = np.clip(np.rint(im), -8, 7).astype(np.int16)
    return (((qr & 0xF) << 4) | (qi & 0xF)).astype(np.uint8)


def random_bytes(rng: np.random.Generator, shape) -> np.ndarray:
    """Uniformly random ci4 bytes (every nibble value equally likely)."""
    return rng.integers(0, 256, size=shape, dtype=np.uint8)


def complex_kernels(seed: int, n_chan: int, n_ant: int, support: int,
                    width_cells: float = 1.5) -> np.ndarray:
    """Seeded complex gridding kernels [C, A, K, K] (complex64) with the shape of
    per-antenna illumination patterns: a smooth envelope of the given width in
    cells, a per-antenna amplitude in [0.7, 1.3], and a per-(channel, antenna)
    phase offset and linear phase gradient across the footprint."""
    rng = np.random.default_rng(seed)
    h = support // 2
    d = np.arange(-h, h + 1, dtype=np.float64)
    env = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * width_cells ** 2))   # [dj, di]
    amp = rng.uniform(0.7, 1.3, size=(1, n_ant, 1, 1))
    ph0 = rng.uniform(0, 2 * np.pi, size=(n_chan, n_ant, 1, 1))
    gj = rng.uniform(-0.6, 0.6, size=(n_chan, n_ant, 1, 1))
    gi = rng.uniform(-0.6, 0.6, size=(n_chan, n_ant, 1, 1))
    phase = ph0 + gj * d[None, None, :, None] + gi * d[None, None, None, :]
    return (amp * env[None, None] * np.exp(1j * phase)).astype(np.complex64)


def with_kernels(inp: "Inputs", support: int, seed: int, width_cells: float = 1.5) -> "Inputs":
    """The same problem gridded with seeded complex kernels of the given support."""
    k = complex_kernels(seed, inp.n_chan, inp.n_ant, support, width_cells)
    return dataclasses.replace(inp, kernel_support=support, kernels=k,
                               name=f"{inp.name}_k{support}c")


def raw_gulp(seed: int, n_time: int, c_in: int, n_ant: int, n_pol: int) -> np.ndarray:
    """Random 4+4-bit bytes in the order they arrive from the channeliser,
    [Time, Channel, Antenna, Polarisation] (no imaging arithmetic: just bytes)."""
    return random_bytes(np.random.default_rng(seed), (n_time, c_in, n_ant, n_pol))


# ---------------------------------------------------------------- layouts
def square_layout(rng: np.random.Generator, n_ant: int, side_m: float) -> np.ndarray:
    return rng.uniform(-side_m / 2, side_m / 2, size=(n_ant, 2))


def disk_layout(rng: np.random.Generator, n_ant: int, diameter_m: float,
                min_sep_m: float, max_darts: int = 2_000_000) -> np.ndarray:
    """Random sequential addition ("dart throwing") inside a disk."""
    r2 = (diameter_m / 2) ** 2
    pts: List[np.ndarray] = []
    arr = np.empty((0, 2))
    tried = 0
    sep2 = min_sep_m * min_sep_m
    while len(pts) < n_ant and tried < max_darts:
        cand = rng.uniform(-diameter_m / 2, diameter_m / 2, size=(4096, 2))
        cand = cand[(cand ** 2).sum(1) <= r2]
        for c in cand:
            tried += 1
            if arr.shape[0] == 0 or ((arr - c) ** 2).sum(1).min() >= sep2:
                pts.append(c)
                arr = np.asarray(pts)
                if len(pts) == n_ant:
                    break
            if tried >= max_darts:
                break
    if len(pts) < n_ant:
        raise RuntimeError(f"disk layout: placed {len(pts)}/{n_ant} antennas "
                           f"with min separation {min_sep_m} m")
    return np.asarray(pts, dtype=np.float64)


def random_gains(rng: np.random.Generator, shape, amp=(0.8, 1.2)) -> np.ndarray:
    a = rng.uniform(amp[0], amp[1], size=shape)
    ph = rng.uniform(0.0, 2 * np.pi, size=shape)
    return (a * np.exp(1j * ph)).astype(np.complex64)


def lwa_channels(n_chan: int, centre_hz: float = 38e6) -> np.ndarray:
    c = np.arange(n_chan, dtype=np.float64)
    return centre_hz + (c - (n_chan - 1) / 2.0) * CHAN_BW_HZ


def on_pixel_direction(rng: np.random.Generator, grid_n: int, cell_wavelengths: float,
                       max_abs: float = 0.7):
    """A direction (l, m) that falls exactly on a pixel centre."""
    step = 1.0 / (grid_n * cell_wavelengths)       # pixel pitch in l, m
    qmax = int(np.floor(max_abs / step))
    ql, qm = rng.integers(-qmax, qmax + 1, size=2)
    return float(ql * step), float(qm * step)


# ---------------------------------------------------------------- sky model
def simulate_efield(rng_sky: np.random.Generator, rng_noise: np.random.Generator,
                    xy_m: np.ndarray, freq_hz: np.ndarray, n_time: int, n_pol: int,
                    src_lm: np.ndarray, src_amp: np.ndarray, src_polfrac: np.ndarray,
                    noise_sigma: float, divide_gains: Optional[np.ndarray] = None,
                    chunk: int = 8) -> np.ndarray:
    """Point sources + Gaussian receiver noise -> packed bytes [T, C, P, A].

    src_amp[k] is the per-antenna amplitude of source k; src_polfrac[k] is the
    correlation between its X and Y time series (0 = unpolarised).
    If divide_gains [C, P, A] is given the sky signal is divided by it before
    quantisation (the corrupted data a gain g_true would calibrate).
    """
    C = freq_hz.shape[0]
    A = xy_m.shape[0]
    K = src_lm.shape[0]
    out = np.empty((n_time, C, n_pol, A), dtype=np.uint8)
    for c0 in range(0, C, chunk):
        c1 = min(C, c0 + chunk)
        lam = C0 / freq_hz[c0:c1]                                  # [c]
        u = xy_m[None, :, 0] / lam[:, None]                        # [c, A]
        v = xy_m[None, :, 1] / lam[:, None]
        sig = np.zeros((n_time, c1 - c0, n_pol, A), dtype=np.complex64)
        for k in range(K):
            ph = np.exp(-2j * np.pi * (u * src_lm[k, 0] + v * src_lm[k, 1]))  # [c, A]
            sx = np.exp(1j * rng_sky.uniform(0, 2 * np.pi, size=(n_time, c1 - c0)))
            series = [sx]
            if n_pol == 2:
                si = np.exp(1j * rng_sky.uniform(0, 2 * np.pi, size=(n_time, c1 - c0)))
                f = float(src_polfrac[k])
                series.append(f * sx + np.sqrt(1.0 - f * f) * si)
            for p in range(n_pol):
                sig[:, :, p, :] += (src_amp[k] * series[p][:, :, None] * ph[None, :, :]).astype(np.complex64)
        if divide_gains is not None:
            sig /= divide_gains[None, c0:c1, :, :]
        noise_re = rng_noise.normal(0.0, noise_sigma, size=sig.shape).astype(np.float32)
        noise_im = rng_noise.normal(0.0, noise_sigma, size=sig.shape).astype(np.float32)
        out[:, c0:c1] = pack_ci4(sig.real + noise_re, sig.imag + noise_im)
    return out


# ---------------------------------------------------------------- presets
def config1(k: int = 1, n_time: int = 8, unity_gains: bool = False,
            noise_sigma: float = 2.0) -> Inputs:
    """Tiny single-pol case: 16 antennas in a 20 m square, 1 channel at 50 MHz,
    32x32 grid at lambda/2, 3x3 Gaussian (sigma 0.5 cell), one unit plane wave."""
    r_lay = np.random.default_rng(1000 + k)
    r_gain = np.random.default_rng(2000 + k)
    r_sky = np.random.default_rng(3000 + k)
    r_noise = np.random.default_rng(4000 + k)
    N, A, P, C = 32, 16, 1, 1
    xy = square_layout(r_lay, A, 20.0)
    freq = np.array([50e6])
    gains = np.ones((C, P, A), np.complex64) if unity_gains else random_gains(r_gain, (C, P, A))
    l0, m0 = on_pixel_direction(r_sky, N, 0.5)
    lm = np.array([[l0, m0]])
    ef = simulate_efield(r_sky, r_noise, xy, freq, n_time, P, lm, np.array([1.0]),
                         np.array([0.0]), noise_sigma)
    return Inputs(N, C, P, A, 3, 0.5, 0.5, xy, freq, gains, ef,
                  sources=dict(lm=lm, amp=np.array([1.0])), name="cfg1")


def config2(k: int = 2, n_time: int = 1000, n_chan: int = 132,
            min_sep_m: float = 4.5) -> Inputs:
    """LWA-like: 256 dual-pol antennas in a 100 m disk, 132 x 25 kHz channels at
    38 MHz, 64x64 grid, 5 point sources with image contrast 1-10 x noise.

    5 m minimum separation is not reachable by random sequential addition for
    256 antennas in a 100 m disk (it jams near 230); 4.5 m is used instead."""
    r_lay = np.random.default_rng(1000 + k)
    r_gain = np.random.default_rng(2000 + k)
    r_sky = np.random.default_rng(3000 + k)
    r_noise = np.random.default_rng(4000 + k)
    N, A, P = 64, 256, 2
    xy = disk_layout(r_lay, A, 100.0, min_sep_m)
    freq = lwa_channels(n_chan)
    gains = random_gains(r_gain, (n_chan, P, A))
    sigma = 2.0
    nsrc = 5
    lm = np.stack([_disk_direction(r_sky, 0.8) for _ in range(nsrc)])
    flux = r_sky.uniform(1.0, 10.0, size=nsrc)
    # image-plane contrast: A^2 p_k = F_k * A * 2 sigma^2  ->  p_k = F_k 2 sigma^2 / A
    amp = np.sqrt(flux * 2 * sigma * sigma / A)
    polfrac = np.zeros(nsrc)
    polfrac[0] = 0.5
    ef = simulate_efield(r_sky, r_noise, xy, freq, n_time, P, lm, amp, polfrac, sigma)
    return Inputs(N, n_chan, P, A, 3, 0.5, 0.5, xy, freq, gains, ef,
                  sources=dict(lm=lm, amp=amp, flux=flux, polfrac=polfrac), name="cfg2")


def config3(k: int = 3, n_time: int = 100_000) -> Inputs:
    """Config-1 geometry and statistics over a long integration."""
    base = config1(k=k, n_time=n_time)
    base.name = "cfg3"
    return base


CONFIG4_BLOCKS = ((32, 64, 264), (32, 64, 16), (64, 256, 132),
                  (64, 256, 40), (128, 1024, 64), (128, 1024, 16))


def config4_block(b: int, k: int = 4, n_time: int = 200, n_pol: int = 2,
                  blocks=CONFIG4_BLOCKS) -> Inputs:
    """One block of the heterogeneous batch: disk diameter N/2 - K cells at the
    block's highest channel, minimum separation 1 cell."""
    N, A, C = blocks[b]
    r_lay = np.random.default_rng(1000 + 10 * k + b)
    r_gain = np.random.default_rng(2000 + 10 * k + b)
    r_sky = np.random.default_rng(3000 + 10 * k + b)
    r_noise = np.random.default_rng(4000 + 10 * k + b)
    freq = lwa_channels(C)
    lam_min = C0 / freq.max()
    cell_m = 0.5 * lam_min
    diam_m = (N / 2 - 3) * cell_m
    xy = disk_layout(r_lay, A, diam_m, cell_m)
    gains = random_gains(r_gain, (C, n_pol, A))
    sigma = 2.0
    lm = np.stack([_disk_direction(r_sky, 0.8) for _ in range(3)])
    flux = r_sky.uniform(1.0, 10.0, size=3)
    amp = np.sqrt(flux * 2 * sigma * sigma / A)
    ef = simulate_efield(r_sky, r_noise, xy, freq, n_time, n_pol, lm, amp,
                         np.zeros(3), sigma)
    return Inputs(N, C, n_pol, A, 3, 0.5, 0.5, xy, freq, gains, ef,
                  sources=dict(lm=lm, amp=amp), name=f"cfg4b{b}")


def config5(k: int = 5, n_time: int = 200, n_chan: int = 64, n_src: int = 20,
            perturb: float = 0.1, min_sep_m: float = 4.5) -> Inputs:
    """Calibration case: true gains per (pol, antenna) shared over channels;
    the data are the sky divided by the true gains; the gains handed to the
    imager are g_true * (1 + perturb * z) with z complex normal.

    sources carries g_true [P, A] and the model sky for the loss."""
    r_lay = np.random.default_rng(1000 + k)
    r_gain = np.random.default_rng(2000 + k)
    r_sky = np.random.default_rng(3000 + k)
    r_noise = np.random.default_rng(4000 + k)
    N, A, P = 64, 256, 2
    xy = disk_layout(r_lay, A, 100.0, min_sep_m)
    freq = 38e6 + np.linspace(-0.8e6, 0.8e6, n_chan)
    g_true = random_gains(r_gain, (P, A)).astype(np.complex128)
    z = (r_gain.normal(size=(P, A)) + 1j * r_gain.normal(size=(P, A))) / np.sqrt(2)
    g_eval = (g_true * (1.0 + perturb * z)).astype(np.complex64)
    sigma = 2.0
    lm = np.stack([_disk_direction(r_sky, 0.8) for _ in range(n_src)])
    flux = r_sky.uniform(1.0, 10.0, size=n_src)
    amp = np.sqrt(flux * 2 * sigma * sigma / A)
    divide = np.broadcast_to(g_true[None], (n_chan, P, A))
    ef = simulate_efield(r_sky, r_noise, xy, freq, n_time, P, lm, amp, np.zeros(n_src),
                         sigma, divide_gains=divide)
    gains = np.broadcast_to(g_eval[None], (n_chan, P, A)).copy()
    return Inputs(N, n_chan, P, A, 3, 0.5, 0.5, xy, freq, gains, ef,
                  sources=dict(lm=lm, amp=amp, flux=flux, g_true=g_true.astype(np.complex64),
                               g_eval=g_eval, noise_sigma=sigma),
                  name="cfg5")


def deployment(seed: int = 50, n_time: int = 1250, n_chan: int = 4, n_pol: int = 2) -> Inputs:
    """The deployed geometry of the paper (Sec. 4.1-4.2): 256 antennas uniform in
    a 110 m x 100 m ellipse elongated north-south, 25 kHz channels centred on
    55.25 MHz, a 64-cell grid at lambda / 2 (about 43 cells across with the
    taps), 3 x 3 Gaussian; random gains and uniformly random bytes.  The
    default n_time is one 50 ms image of 40 us samples."""
    rng = np.random.default_rng(seed)
    A = 256
    r = np.sqrt(rng.uniform(0.0, 1.0, A))
    t = rng.uniform(0.0, 2 * np.pi, A)
    xy = np.stack([50.0 * r * np.cos(t), 55.0 * r * np.sin(t)], 1)
    freq = lwa_channels(n_chan, 55.25e6)
    gains = random_gains(rng, (n_chan, n_pol, A))
    ef = random_bytes(rng, (n_time, n_chan, n_pol, A))
    return Inputs(64, n_chan, n_pol, A, 3, 0.5, 0.5, xy, freq, gains, ef, name=f"deployment{seed}")


def random_problem(seed: int, grid_n: int, n_ant: int, n_chan: int, n_pol: int,
                   n_time: int, centre_hz: float = 38e6, fill: float = 0.45,
                   min_sep_cells: float = 1.0) -> Inputs:
    """Generic seeded case for parity sweeps: disk layout that fits the grid at the
    highest channel, random gains, uniformly random bytes."""
    rng = np.random.default_rng(seed)
    freq = lwa_channels(n_chan, centre_hz)
    lam_min = C0 / freq.max()
    cell_m = 0.5 * lam_min
    diam_m = max(2.0, (fill * grid_n - 3) * cell_m)
    xy = disk_layout(rng, n_ant, diam_m, min_sep_cells * cell_m * 0.5) if n_ant > 1 \
        else rng.uniform(-diam_m / 4, diam_m / 4, size=(1, 2))
    gains = random_gains(rng, (n_chan, n_pol, n_ant))
    ef = random_bytes(rng, (n_time, n_chan, n_pol, n_ant))
    return Inputs(grid_n, n_chan, n_pol, n_ant, 3, 0.5, 0.5, xy, freq, gains, ef,
                  name=f"rand{seed}")


def _disk_direction(rng: np.random.Generator, rmax: float):
    while True:
        l, m = rng.uniform(-rmax, rmax, size=2)
        if l * l + m * m <= rmax * rmax:
            return np.array([l, m])
