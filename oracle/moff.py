"""Plain FP64 CPU oracle of the MOFF direct-imaging hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; it exists so that tests/, the smoke check and the benchmark's CPU
baseline can check the GPU library against an implementation that is slow,
double precision and obviously correct.  It shares no code with the GPU path.

What it computes (Kent et al. 2019, "A Real-Time, All-Sky, High Time
Resolution, Direct Imager for the Long Wavelength Array"):

  * §3.2: channelised 4+4-bit complex E-fields ordered [T, C, P, A] are
    unpacked to complex numbers and multiplied by a per-antenna complex
    calibration factor (delay calibration / gain);
  * §2.1 Eq. (4)-(5): each antenna's point measurement E' is convolved with an
    illumination kernel W and gridded onto a regular aperture grid with a
    spacing of half the channel wavelength (§3.2, §4.2);
  * §2.1 Eq. (5), §3.2: the gridded aperture is spatially Fourier transformed
    with the +i sign ("inverse" transform), unnormalised;
  * §2.1 Eq. (5), §3.2: the image is squared, or cross multiplied between the
    two polarisations (XX, XY, YX, YY), and accumulated (summed) over time.

Readings where the paper is silent (each is listed with its reason in the
design notes of the repository):
  * nibble order: high nibble = real part, low nibble = imaginary part, two's
    complement in [-8, 7];
  * gains g[c, p, a] multiply the E-field; delays are a phase inside g;
  * aperture centred on the grid: X = x / (lambda_c * du) + N/2 (cells);
  * kernel = exact Gaussian of width sigma (cells) evaluated at each tap's
    offset from the antenna, peak 1, no renormalisation, support K x K
    centred on the nearest cell (ties round up: floor(X + 1/2));
  * a tap outside [0, N) is an error (no wrap, no clipping);
  * transform F[km, kl] = sum_{j,i} A[j, i] exp(+2 pi i (i kl + j km) / N),
    rows j <-> y / m, columns i <-> x / l;
  * XY = F_X conj(F_Y), YX = F_Y conj(F_X); "accumulated" = sum over T;
  * output pixels fftshifted on both axes: pixel q <-> l = (q - N/2) / (N du).
"""
from __future__ import annotations

import numpy as np

C0 = 299_792_458.0


class OffGridError(ValueError):
    """A kernel tap of some antenna falls outside the grid for some channel."""


# ------------------------------------------------------------ front end (§3.2)
def decimate_transpose(raw: np.ndarray, n_chan: int, c0: int = 0, c_step: int = 1) -> np.ndarray:
    """The front end before imaging (§3.2): channelised bytes arriving as
    [Time, Channel, Antenna, Polarisation] are decimated in frequency (output
    channel i is input channel c0 + i * c_step) and transposed to
    [Time, Channel, Polarisation, Antenna].  Bytes are moved, never changed."""
    raw = np.asarray(raw)
    T, c_in, A, P = raw.shape
    if c0 < 0 or c_step < 1 or n_chan < 1 or c0 + (n_chan - 1) * c_step >= c_in:
        raise ValueError("channel selection outside the input")
    sel = raw[:, c0:c0 + (n_chan - 1) * c_step + 1:c_step]           # [T, C, A, P]
    return np.ascontiguousarray(np.transpose(sel, (0, 1, 3, 2)))


# --------------------------------------------------------------------- O1
def unpack_ci4(b: np.ndarray) -> np.ndarray:
    """4+4-bit complex integers -> complex128 (§3.2: "4+4-bit complex integer").

    High nibble = real part, low nibble = imaginary part, each two's complement.
    """
    v = np.asarray(b).astype(np.int64)
    hi = v >> 4
    lo = v & 0xF
    re = np.where(hi >= 8, hi - 16, hi)
    im = np.where(lo >= 8, lo - 16, lo)
    return re.astype(np.float64) + 1j * im.astype(np.float64)


# --------------------------------------------------------------------- O3
def antenna_cells(xy_m: np.ndarray, freq_hz: np.ndarray, grid_n: int,
                  cell_wavelengths: float = 0.5):
    """Antenna positions in grid-cell units per channel (§3.2, §4.2: grid spacing
    of half the channel wavelength).  Returns X, Y of shape [C, A]."""
    xy = np.asarray(xy_m, dtype=np.float64)
    f = np.asarray(freq_hz, dtype=np.float64)
    if not np.all(np.isfinite(xy)):
        raise ValueError("antenna positions must be finite")
    if not (np.all(np.isfinite(f)) and np.all(f > 0)):
        raise ValueError("channel frequencies must be finite and positive")
    lam = C0 / f                                   # metres, [C]
    cell_m = lam * cell_wavelengths                # metres per cell, [C]
    X = xy[None, :, 0] / cell_m[:, None] + grid_n / 2.0
    Y = xy[None, :, 1] / cell_m[:, None] + grid_n / 2.0
    return X, Y


def kernel_taps(X: np.ndarray, Y: np.ndarray, grid_n: int, support: int = 3,
                sigma_cells: float = 0.5, kernels=None):
    """Cells and weights of the illumination kernel W around each antenna
    (§2.1 Eq. (4): E = W * E').  Returns ii, jj (int) and w, each of shape
    [C, A, K*K], tap order (dj outer, di inner).

    kernels None: w = the Gaussian of width sigma_cells at each tap's offset
    (float64).  Otherwise kernels [C, A, K, K] (complex) gives each channel's
    and antenna's own kernel on the same K x K cells (§3.3: any kernel per
    antenna, e.g. its illumination pattern for A-projection); w = kernels."""
    if support < 1 or support % 2 == 0:
        raise ValueError("kernel support must be odd and positive")
    if kernels is None and not sigma_cells > 0:
        raise ValueError("kernel width must be positive")
    h = support // 2
    i0 = np.floor(X + 0.5).astype(np.int64)
    j0 = np.floor(Y + 0.5).astype(np.int64)
    d = np.arange(-h, h + 1)
    dj, di = np.meshgrid(d, d, indexing="ij")      # dj outer, di inner
    di = di.reshape(-1)
    dj = dj.reshape(-1)
    ii = i0[..., None] + di
    jj = j0[..., None] + dj
    if kernels is None:
        w = np.exp(-((ii - X[..., None]) ** 2 + (jj - Y[..., None]) ** 2)
                   / (2.0 * sigma_cells ** 2))
    else:
        kern = np.asarray(kernels)
        if kern.shape != X.shape + (support, support):
            raise ValueError(f"kernels must be [C, A, {support}, {support}]")
        w = kern.astype(np.complex128).reshape(X.shape + (support * support,))
    if ii.min() < 0 or jj.min() < 0 or ii.max() >= grid_n or jj.max() >= grid_n:
        raise OffGridError("a kernel tap falls outside the grid")
    return ii, jj, w


# --------------------------------------------------------------------- O4
def grid_efield(eprime: np.ndarray, ii: np.ndarray, jj: np.ndarray,
                w: np.ndarray, grid_n: int) -> np.ndarray:
    """Gridded aperture A = W * E' for one channel (§2.1 Eq. (5)).

    eprime [T, P, A] complex; ii, jj, w [A, K*K].  Overlapping footprints add.
    Returns [T, P, N, N] with A[t, p, j, i] (row j <-> y, column i <-> x)."""
    T, P, Aant = eprime.shape
    out = np.zeros((T, P, grid_n, grid_n), dtype=np.complex128)
    for a in range(Aant):
        for k in range(ii.shape[1]):
            out[:, :, jj[a, k], ii[a, k]] += w[a, k] * eprime[:, :, a]
    return out


# --------------------------------------------------------------------- O5
def transform(agrid: np.ndarray) -> np.ndarray:
    """Unnormalised +i 2-D DFT over the last two axes (§2.1 Eq. (5); §3.2
    "inverse Fourier transformed"): F[km, kl] = sum A[j, i] e^{+2 pi i (i kl + j km)/N}."""
    n = agrid.shape[-1] * agrid.shape[-2]
    return np.fft.ifft2(agrid, axes=(-2, -1)) * n


def direct_dft(agrid: np.ndarray) -> np.ndarray:
    """The same transform evaluated straight from its definition, O(n_g^2)."""
    N = agrid.shape[-1]
    k = np.arange(N)
    phase = np.exp(2j * np.pi * np.outer(k, k) / N)          # [k, n]
    out = np.zeros(agrid.shape, dtype=np.complex128)
    for km in range(N):
        for kl in range(N):
            out[..., km, kl] = np.sum(agrid * phase[km][:, None] * phase[kl][None, :],
                                      axis=(-2, -1))
    return out


# --------------------------------------------------------------------- O6
def products(F: np.ndarray) -> np.ndarray:
    """Polarisation products of the instantaneous images (§2.1, §3.2).

    F [T, P, N, N] -> [T, n_prod, N, N]: P = 1 -> (XX,); P = 2 -> (XX, XY, YX, YY)
    with XY = F_X conj(F_Y) and YX = F_Y conj(F_X)."""
    def power(f):                      # |f|^2, real by construction
        return (f.real ** 2 + f.imag ** 2).astype(np.complex128)
    if F.shape[1] == 1:
        return power(F[:, 0])[:, None]
    fx, fy = F[:, 0], F[:, 1]
    xy = fx * np.conj(fy)
    return np.stack([power(fx), xy, np.conj(xy), power(fy)], axis=1)


def n_products(n_pol: int) -> int:
    return 1 if n_pol == 1 else 4


# ------------------------------------------------------------ O1..O8 chained
def image(xy_m, freq_hz, gains, efield, grid_n, kernel_support=3,
          kernel_sigma_cells=0.5, cell_wavelengths=0.5, chunk=128, kernels=None) -> np.ndarray:
    """Accumulated polarised images, complex128 [C, n_prod, N, N], fftshifted.

    gains [C, P, A] complex (promoted exactly to complex128);
    efield [T, C, P, A] uint8 (ci4).  Images are summed over all T samples."""
    efield = np.asarray(efield)
    T, C, P, Aant = efield.shape
    X, Y = antenna_cells(xy_m, freq_hz, grid_n, cell_wavelengths)
    ii, jj, w = kernel_taps(X, Y, grid_n, kernel_support, kernel_sigma_cells, kernels)
    g = np.asarray(gains).astype(np.complex128)
    out = np.zeros((C, n_products(P), grid_n, grid_n), dtype=np.complex128)
    for c in range(C):
        acc = np.zeros((n_products(P), grid_n, grid_n), dtype=np.complex128)
        for t0 in range(0, T, chunk):
            e = unpack_ci4(efield[t0:t0 + chunk, c])                 # [t, P, A]
            eprime = g[c][None] * e                                  # O2
            F = transform(grid_efield(eprime, ii[c], jj[c], w[c], grid_n))
            prods = products(F)
            for t in range(prods.shape[0]):                          # O7, in time order
                acc += prods[t]
        out[c] = np.fft.fftshift(acc, axes=(-2, -1))                 # O8
    return out


def image_from(inp, **kw) -> np.ndarray:
    """image() on a synth.Inputs-like object (anything with the same fields)."""
    kw.setdefault("kernels", getattr(inp, "kernels", None))
    return image(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, inp.grid_n,
                 inp.kernel_support, inp.kernel_sigma_cells, inp.cell_wavelengths, **kw)


# --------------------------------------------------------------- FX form (P5)
def aperture_response(xy_m, freq_hz, grid_n, kernel_support=3, kernel_sigma_cells=0.5,
                      cell_wavelengths=0.5, kernels=None) -> np.ndarray:
    """b[c, a, km, kl] = sum_taps w e^{+2 pi i (i kl + j km)/N}: the transform of
    one antenna's kernel footprint (unshifted pixel order)."""
    X, Y = antenna_cells(xy_m, freq_hz, grid_n, cell_wavelengths)
    ii, jj, w = kernel_taps(X, Y, grid_n, kernel_support, kernel_sigma_cells, kernels)
    N = grid_n
    k = np.arange(N)
    C, Aant, KK = w.shape
    b = np.zeros((C, Aant, N, N), dtype=np.complex128)
    for t in range(KK):
        pl = np.exp(2j * np.pi * ii[..., t, None] * k[None, None, :] / N)    # [C, A, kl]
        pm = np.exp(2j * np.pi * jj[..., t, None] * k[None, None, :] / N)    # [C, A, km]
        b += w[..., t, None, None] * pm[..., :, None] * pl[..., None, :]
    return b


def visibilities(gains, efield) -> np.ndarray:
    """V_PQ[c, a, b] = sum_t e'_{P,a} conj(e'_{Q,b}) (§2 Eq. (2)), complex128
    [C, n_prod, A, A] in product order XX, XY, YX, YY."""
    e = unpack_ci4(efield)                                           # [T, C, P, A]
    ep = np.asarray(gains).astype(np.complex128)[None] * e
    P = ep.shape[2]
    pairs = [(0, 0)] if P == 1 else [(0, 0), (0, 1), (1, 0), (1, 1)]
    return np.stack([np.einsum("tca,tcb->cab", ep[:, :, p], np.conj(ep[:, :, q]))
                     for p, q in pairs], axis=1)


def image_fx(xy_m, freq_hz, gains, efield, grid_n, kernel_support=3,
             kernel_sigma_cells=0.5, cell_wavelengths=0.5, vis=None, kernels=None) -> np.ndarray:
    """The same accumulated image from visibilities (the FX route, §2 Eq. (1)-(2)):
    I_PQ(k) = sum_{a,b} V_PQ[a,b] b_a(k) conj(b_b(k)).  No gridding, no FFT."""
    b = aperture_response(xy_m, freq_hz, grid_n, kernel_support, kernel_sigma_cells,
                          cell_wavelengths, kernels)                  # [C, A, N, N]
    V = visibilities(gains, efield) if vis is None else vis          # [C, n, A, A]
    C = b.shape[0]
    N = grid_n
    bf = b.reshape(C, b.shape[1], N * N)
    out = np.einsum("ckab,cap,cbp->ckp", V, bf, np.conj(bf))
    return np.fft.fftshift(out.reshape(C, V.shape[1], N, N), axes=(-2, -1))


# ------------------------------------------- autocorrelation removal (§3.2)
def auto_visibilities(gains, efield) -> np.ndarray:
    """The antenna autocorrelations V_PQ[c, a, a] = sum_t e'_{P,a} conj(e'_{Q,a})
    (the a = b entries of §2 Eq. (2)), complex128 [C, n_prod, A], products in
    the order XX, XY, YX, YY."""
    e = unpack_ci4(efield)                                           # [T, C, P, A]
    ep = np.asarray(gains).astype(np.complex128)[None] * e
    P = ep.shape[2]
    pairs = [(0, 0)] if P == 1 else [(0, 0), (0, 1), (1, 0), (1, 1)]
    return np.stack([np.sum(ep[:, :, p] * np.conj(ep[:, :, q]), axis=0) for p, q in pairs], axis=1)


def autocorrelation_image(xy_m, freq_hz, gains, efield, grid_n, kernel_support=3,
                          kernel_sigma_cells=0.5, cell_wavelengths=0.5, kernels=None) -> np.ndarray:
    """The zero-spacing part of the accumulated image that §3.2 optionally
    removes: the a = b terms sum_a V_PQ[a, a] |b_a(k)|^2 of the visibility form
    (fftshifted, like the image)."""
    b = aperture_response(xy_m, freq_hz, grid_n, kernel_support, kernel_sigma_cells,
                          cell_wavelengths, kernels)                  # [C, A, N, N]
    vd = auto_visibilities(gains, efield)                            # [C, n, A]
    out = np.einsum("cka,cayx->ckyx", vd, np.abs(b) ** 2)
    return np.fft.fftshift(out, axes=(-2, -1))


def image_without_autos(xy_m, freq_hz, gains, efield, grid_n, kernel_support=3,
                        kernel_sigma_cells=0.5, cell_wavelengths=0.5, kernels=None) -> np.ndarray:
    """The accumulated image with the antenna autocorrelations removed (§3.2):
    image minus autocorrelation_image."""
    full = image(xy_m, freq_hz, gains, efield, grid_n, kernel_support, kernel_sigma_cells,
                 cell_wavelengths, kernels=kernels)
    return full - autocorrelation_image(xy_m, freq_hz, gains, efield, grid_n, kernel_support,
                                        kernel_sigma_cells, cell_wavelengths, kernels)


def image_without_autos_from(inp) -> np.ndarray:
    return image_without_autos(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, inp.grid_n,
                               inp.kernel_support, inp.kernel_sigma_cells, inp.cell_wavelengths,
                               getattr(inp, "kernels", None))


# ------------------------------------------------------------- O9 gradient
def grad_gains(xy_m, freq_hz, gains, efield, grid_n, grad_image, kernel_support=3,
               kernel_sigma_cells=0.5, cell_wavelengths=0.5, chunk=128, kernels=None) -> np.ndarray:
    """d(loss)/d(gain) in the PyTorch complex convention (dL/dRe + i dL/dIm),
    given grad_image = dL/dRe(I) + i dL/dIm(I) in the image layout.

    Wirtinger chain (F = Phi A with Phi the +i DFT; A = sum w e' is holomorphic
    in g, so the kernel enters conjugated):
      dL/dF_X* = Re(G_XX) F_X + h F_Y,  dL/dF_Y* = Re(G_YY) F_Y + conj(h) F_X,
      h = (G_XY + conj(G_YX)) / 2;  dL/dA* = Phi^H dL/dF*  (the -i transform);
      dL/dg*[c,p,a] = sum_t sum_taps conj(w) conj(e[t,c,p,a]) (dL/dA*)[tap];
      returned gradient = 2 dL/dg*.
    The imaginary parts of G_XX, G_YY are ignored: those products are real."""
    efield = np.asarray(efield)
    T, C, P, Aant = efield.shape
    N = grid_n
    X, Y = antenna_cells(xy_m, freq_hz, N, cell_wavelengths)
    ii, jj, w = kernel_taps(X, Y, N, kernel_support, kernel_sigma_cells, kernels)
    g = np.asarray(gains).astype(np.complex128)
    Gam = np.fft.ifftshift(np.asarray(grad_image).astype(np.complex128), axes=(-2, -1))
    out = np.zeros((C, P, Aant), dtype=np.complex128)
    for c in range(C):
        a_xx = Gam[c, 0].real
        if P == 2:
            a_yy = Gam[c, 3].real
            h = 0.5 * (Gam[c, 1] + np.conj(Gam[c, 2]))
        for t0 in range(0, T, chunk):
            e = unpack_ci4(efield[t0:t0 + chunk, c])                  # [t, P, A]
            F = transform(grid_efield(g[c][None] * e, ii[c], jj[c], w[c], N))
            if P == 1:
                G = (a_xx * F[:, 0])[:, None]
            else:
                gx = a_xx * F[:, 0] + h * F[:, 1]
                gy = a_yy * F[:, 1] + np.conj(h) * F[:, 0]
                G = np.stack([gx, gy], axis=1)
            H = np.fft.fft2(G, axes=(-2, -1))                          # Phi^H, unnormalised
            Htap = H[:, :, jj[c], ii[c]]                                # [t, P, A, K*K]
            out[c] += np.einsum("ak,tpak,tpa->pa", np.conj(w[c]), Htap, np.conj(e))
    return 2.0 * out


def grad_autos(xy_m, freq_hz, gains, efield, grid_n, grad_image, kernel_support=3,
               kernel_sigma_cells=0.5, cell_wavelengths=0.5, kernels=None) -> np.ndarray:
    """The share of autocorrelation_image in the gain gradient: d/dg of
    Re <grad_image, autocorrelation_image>, in the convention of grad_gains.

    With B_a(k) = |b_a(k)|^2 (real), s_PQ[a] = sum_t e_P conj(e_Q) (no gains) and
    U_PQ[a] = sum_k Gamma_PQ(k) B_a(k):
      V_XX = |g_X|^2 s_XX           ->  2 Re(U_XX) s_XX g_X
      V_XY = g_X conj(g_Y) s_XY, V_YX = conj(V_XY), H = U_XY + conj(U_YX)
                                    ->  H conj(s_XY) g_Y  to X,  conj(H) s_XY g_X  to Y
    (the imaginary parts of Gamma_XX, Gamma_YY are ignored, as in grad_gains)."""
    b = aperture_response(xy_m, freq_hz, grid_n, kernel_support, kernel_sigma_cells,
                          cell_wavelengths, kernels)
    B = np.abs(b) ** 2                                                # [C, A, N, N]
    Gam = np.fft.ifftshift(np.asarray(grad_image).astype(np.complex128), axes=(-2, -1))
    e = unpack_ci4(efield)                                            # [T, C, P, A]
    g = np.asarray(gains).astype(np.complex128)
    P = e.shape[2]
    out = np.zeros(g.shape, dtype=np.complex128)
    s_xx = np.sum(np.abs(e[:, :, 0]) ** 2, axis=0)                   # [C, A]
    u_xx = np.einsum("cyx,cayx->ca", Gam[:, 0].real, B)
    out[:, 0] = 2.0 * u_xx * s_xx * g[:, 0]
    if P == 2:
        s_yy = np.sum(np.abs(e[:, :, 1]) ** 2, axis=0)
        s_xy = np.sum(e[:, :, 0] * np.conj(e[:, :, 1]), axis=0)
        u_yy = np.einsum("cyx,cayx->ca", Gam[:, 3].real, B)
        h = np.einsum("cyx,cayx->ca", Gam[:, 1] + np.conj(Gam[:, 2]), B)
        out[:, 0] += h * np.conj(s_xy) * g[:, 1]
        out[:, 1] = 2.0 * u_yy * s_yy * g[:, 1] + np.conj(h) * s_xy * g[:, 0]
    return out


def grad_gains_without_autos(xy_m, freq_hz, gains, efield, grid_n, grad_image,
                             kernel_support=3, kernel_sigma_cells=0.5,
                             cell_wavelengths=0.5, kernels=None) -> np.ndarray:
    """Gain gradient of a loss of image_without_autos: grad_gains minus grad_autos."""
    args = (xy_m, freq_hz, gains, efield, grid_n, grad_image, kernel_support,
            kernel_sigma_cells, cell_wavelengths)
    return grad_gains(*args, kernels=kernels) - grad_autos(*args, kernels=kernels)


# ------------------------------------------------------------- losses, FD
def l2_loss(img: np.ndarray, model: np.ndarray) -> float:
    """L = sum over channels, products and pixels of |I - M|^2."""
    d = img - model
    return float(np.sum(d.real ** 2 + d.imag ** 2))


def l2_loss_grad_image(img: np.ndarray, model: np.ndarray) -> np.ndarray:
    """dL/dRe(I) + i dL/dIm(I) for l2_loss: 2 (I - M)."""
    return 2.0 * (img - model)


def fd_grad(loss_of_gains, gains, coords, rel_step=1e-6):
    """Central finite differences on Re g and Im g separately (FP64).

    coords: iterable of index tuples into gains.  Returns complex array
    dL/dRe g + i dL/dIm g at those coordinates."""
    g0 = np.asarray(gains).astype(np.complex128)
    out = []
    for idx in coords:
        hstep = rel_step * max(1.0, abs(g0[idx]))
        parts = []
        for unit in (1.0, 1j):
            gp = g0.copy()
            gm = g0.copy()
            gp[idx] += unit * hstep
            gm[idx] -= unit * hstep
            parts.append((loss_of_gains(gp) - loss_of_gains(gm)) / (2 * hstep))
        out.append(parts[0] + 1j * parts[1])
    return np.asarray(out)


def fd_directional(loss_of_gains, gains, direction, rel_step=1e-6) -> float:
    """Central difference of L along a complex direction d: dL/ds at g + s d."""
    g0 = np.asarray(gains).astype(np.complex128)
    d = np.asarray(direction).astype(np.complex128)
    hstep = rel_step * max(1.0, float(np.abs(g0).max()))
    return (loss_of_gains(g0 + hstep * d) - loss_of_gains(g0 - hstep * d)) / (2 * hstep)


# ------------------------------------------------------- O11 model image
def model_image(xy_m, freq_hz, grid_n, n_time, src_lm, src_power, noise_sigma,
                n_pol=2, kernel_support=3, kernel_sigma_cells=0.5,
                cell_wavelengths=0.5) -> np.ndarray:
    """FX-form image of model visibilities for unpolarised point sources:
    V = T (sum_k S_k p_k p_k^H + 2 sigma^2 Id), p_{k,a} = exp(-2 pi i (u_a l_k + v_a m_k)),
    XY = YX = 0.  Returns [C, n_prod, N, N] fftshifted."""
    b = aperture_response(xy_m, freq_hz, grid_n, kernel_support, kernel_sigma_cells,
                          cell_wavelengths)                           # [C, A, N, N]
    C, Aant, N, _ = b.shape
    lam = C0 / np.asarray(freq_hz, dtype=np.float64)
    xy = np.asarray(xy_m, dtype=np.float64)
    u = xy[None, :, 0] / lam[:, None]
    v = xy[None, :, 1] / lam[:, None]
    img = np.zeros((C, N, N))
    for k in range(len(src_power)):
        p = np.exp(-2j * np.pi * (u * src_lm[k][0] + v * src_lm[k][1]))   # [C, A]
        resp = np.einsum("ca,camn->cmn", p, b)
        img += src_power[k] * np.abs(resp) ** 2
    img += 2.0 * noise_sigma ** 2 * np.sum(np.abs(b) ** 2, axis=1)
    img *= n_time
    out = np.zeros((C, n_products(n_pol), N, N), dtype=np.complex128)
    out[:, 0] = img
    if n_pol == 2:
        out[:, 3] = img
    return np.fft.fftshift(out, axes=(-2, -1))


# ------------------------------------------------ post-processing (§3.2, §4.3)
def pseudo_stokes(img: np.ndarray) -> np.ndarray:
    """Pseudo-Stokes images from the accumulated products (§4.3: linear
    combinations of the linear-polarisation coherencies, leakage not removed):
    I = XX + YY, Q = XX - YY, U = XY + YX, V = -i (XY - YX), all real.
    img [C, 4, N, N] (XX, XY, YX, YY) -> float64 [C, 4, N, N] (I, Q, U, V);
    one polarisation: [C, 1, N, N] -> XX (real)."""
    img = np.asarray(img)
    if img.shape[1] == 1:
        return img.real.copy()
    xx, xy, yx, yy = img[:, 0], img[:, 1], img[:, 2], img[:, 3]
    return np.stack([(xx + yy).real, (xx - yy).real, (xy + yx).real, (-1j * (xy - yx)).real],
                    axis=1)


def kernel_taper(xy_m, freq_hz, grid_n, kernel_support=3, kernel_sigma_cells=0.5,
                 cell_wavelengths=0.5, kernels=None) -> np.ndarray:
    """The imprint of the gridding kernels on a power image (§3.2: known in
    advance, removable after the fact): the antennas' mean kernel power
    pattern T[c, k] = mean_a |b_a(k)|^2, fftshifted like the image.  When every
    antenna has the same kernel up to a whole-cell shift, each product is the
    product of a point-kernel image and exactly this T."""
    b = aperture_response(xy_m, freq_hz, grid_n, kernel_support, kernel_sigma_cells,
                          cell_wavelengths, kernels)
    return np.fft.fftshift(np.mean(np.abs(b) ** 2, axis=1), axes=(-2, -1))


def taper_corrected(planes: np.ndarray, taper: np.ndarray, floor: float) -> np.ndarray:
    """planes [C, n, N, N] divided by taper [C, N, N] where the taper is at
    least floor times its channel's maximum, zero elsewhere."""
    t = np.asarray(taper, dtype=np.float64)
    keep = t >= floor * t.reshape(t.shape[0], -1).max(axis=1)[:, None, None]
    out = np.zeros(np.shape(planes), dtype=np.float64)
    np.divide(planes, t[:, None], out=out, where=np.broadcast_to(keep[:, None], out.shape))
    return out


# -------------------------------------------------------- error metric
def rel_errors(img: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per (channel, product) relative L2 error.  XX, YY: ||dI|| / ||I_ref||.
    XY, YX: ||dI|| / sqrt(||XX_ref|| ||YY_ref||) (unpolarised skies make XY small)."""
    d = np.linalg.norm((img - ref).reshape(img.shape[0], img.shape[1], -1), axis=-1)
    r = np.linalg.norm(ref.reshape(ref.shape[0], ref.shape[1], -1), axis=-1)
    out = np.empty_like(d)
    if img.shape[1] == 1:
        out[:, 0] = d[:, 0] / np.maximum(r[:, 0], 1e-300)
        return out
    scale_x = np.sqrt(r[:, 0] * r[:, 3])
    out[:, 0] = d[:, 0] / np.maximum(r[:, 0], 1e-300)
    out[:, 3] = d[:, 3] / np.maximum(r[:, 3], 1e-300)
    out[:, 1] = d[:, 1] / np.maximum(scale_x, 1e-300)
    out[:, 2] = d[:, 2] / np.maximum(scale_x, 1e-300)
    return out
