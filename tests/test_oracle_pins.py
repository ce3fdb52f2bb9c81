"""Pins of the FP64 oracle to facts that do not come from the oracle itself:
hand-derived values, closed forms, the definition of the DFT evaluated by brute
force, Parseval, the autocorrelation (van Cittert-Zernike) identity, the
visibility (FX) form of the same image, symmetries and invariances.

Each test names the part of the oracle a plausible mistake would break.
"""
import numpy as np
import pytest

import oracle
import synth

E2 = np.exp(-2.0)       # Gaussian sigma = 0.5 cell, one cell away: exp(-1 / (2 * 0.25))
E4 = np.exp(-4.0)


def _rng(s):
    return np.random.default_rng(s)


# ------------------------------------------------------------------ O1
def test_unpack_byte_table():
    """High nibble = real, low nibble = imaginary, two's complement (hand table)."""
    cases = {0x00: 0 + 0j, 0x7F: 7 - 1j, 0x80: -8 + 0j, 0xF8: -1 - 8j, 0x12: 1 + 2j,
             0x9C: -7 - 4j, 0x08: 0 - 8j, 0x77: 7 + 7j, 0xFF: -1 - 1j, 0x88: -8 - 8j}
    b = np.array(list(cases), dtype=np.uint8)
    got = oracle.unpack_ci4(b)
    assert np.array_equal(got, np.array(list(cases.values())))
    allb = oracle.unpack_ci4(np.arange(256, dtype=np.uint8))
    assert allb.real.min() == -8 and allb.real.max() == 7
    assert allb.imag.min() == -8 and allb.imag.max() == 7
    assert len(set(allb.tolist())) == 256


def test_pack_roundtrip():
    re = np.arange(-8, 8).repeat(16)
    im = np.tile(np.arange(-8, 8), 16)
    b = synth.pack_ci4(re, im)
    e = oracle.unpack_ci4(b)
    assert np.array_equal(e.real, re) and np.array_equal(e.imag, im)


# ------------------------------------------------------------------ O3
def test_geometry_centre_and_scale():
    """lambda/2 cells: an antenna at +one cell east lands one column right of centre."""
    f = np.array([50e6])
    cell = oracle.C0 / 50e6 * 0.5
    xy = np.array([[0.0, 0.0], [cell, 0.0], [0.0, -2 * cell]])
    X, Y = oracle.antenna_cells(xy, f, 32)
    assert np.allclose(X[0], [16, 17, 16], atol=1e-12)
    assert np.allclose(Y[0], [16, 16, 14], atol=1e-12)


def test_kernel_weights_closed_form():
    """On a cell centre: 1, exp(-2), exp(-4); half-cell offsets round up."""
    ii, jj, w = oracle.kernel_taps(np.array([[16.0]]), np.array([[10.0]]), 32)
    expect = np.array([E4, E2, E4, E2, 1.0, E2, E4, E2, E4])
    assert np.allclose(w[0, 0], expect, rtol=1e-14)
    assert list(ii[0, 0]) == [15, 16, 17] * 3
    assert list(jj[0, 0]) == [9] * 3 + [10] * 3 + [11] * 3
    ii, jj, w = oracle.kernel_taps(np.array([[16.5]]), np.array([[10.0]]), 32)
    assert list(ii[0, 0][:3]) == [16, 17, 18]
    wx = np.array([np.exp(-0.5), np.exp(-0.5), np.exp(-4.5)])
    wy = np.array([E2, 1.0, E2])
    assert np.allclose(w[0, 0], np.outer(wy, wx).ravel(), rtol=1e-14)


def test_offgrid_raises():
    with pytest.raises(oracle.OffGridError):
        oracle.kernel_taps(np.array([[0.2]]), np.array([[10.0]]), 32)
    with pytest.raises(oracle.OffGridError):
        oracle.kernel_taps(np.array([[30.6]]), np.array([[10.0]]), 32)
    oracle.kernel_taps(np.array([[1.4]]), np.array([[30.4]]), 32)      # last legal cells


# ------------------------------------------------------------------ P1
@pytest.mark.parametrize("n", [8, 16, 32])
def test_p1_transform_equals_direct_dft(n):
    a = _rng(n).normal(size=(2, n, n)) + 1j * _rng(n + 1).normal(size=(2, n, n))
    f = oracle.transform(a)
    d = oracle.direct_dft(a)
    assert np.linalg.norm(f - d) / np.linalg.norm(d) < 1e-12


def test_p1_transform_sign_single_cell():
    """A single unit cell at (j, i) = (0, 1): F[km, kl] = exp(+2 pi i kl / N)."""
    n = 16
    a = np.zeros((n, n), complex)
    a[0, 1] = 1.0
    f = oracle.transform(a)
    k = np.arange(n)
    assert np.allclose(f, np.exp(2j * np.pi * k / n)[None, :].repeat(n, 0), atol=1e-13)


# ------------------------------------------------------------------ P2
def _on_cell_plane_wave(n_ant, ql, qm, s, n_time=3, seed=0, gains=None):
    """Antennas on whole cells of a 32 grid, a plane wave whose per-antenna phase
    is a multiple of 90 degrees, so its int4 bytes are exact."""
    N = 32
    rng = _rng(seed)
    cell = oracle.C0 / 50e6 * 0.5
    cells = set()
    while len(cells) < n_ant:
        cells.add(tuple(rng.integers(-8, 9, size=2)))
    cxy = np.array(sorted(cells), dtype=float)                  # cells rel. to centre
    xy = cxy * cell
    # exp(-2 pi i (u l0 + v m0)), u l0 = cx * ql / N with l0 = ql / (N du)
    turns = -(cxy[:, 0] * ql + cxy[:, 1] * qm) / N              # multiples of 1/4
    assert np.allclose(turns * 4, np.round(turns * 4))
    ph = np.exp(2j * np.pi * turns)
    e = s * ph
    b = synth.pack_ci4(np.round(e.real), np.round(e.imag))
    ef = np.broadcast_to(b[None, None, None, :], (n_time, 1, 1, n_ant)).copy()
    g = np.ones((1, 1, n_ant), np.complex64) if gains is None else gains
    return xy, np.array([50e6]), g, ef


@pytest.mark.parametrize("ql,qm", [(8, 0), (0, -8), (-8, 8), (8, 8), (0, 0)])
def test_p2_plane_wave_lands_on_its_pixel(ql, qm):
    """Value at the predicted pixel = T |s|^2 A^2 B(k0)^2, where B is the hand-derived
    transform of the 3x3 Gaussian (sigma 1/2 cell):
    B(k) = (1 + 2 e^-2 cos(2 pi kl/N)) (1 + 2 e^-2 cos(2 pi km/N)); and the
    image divided by B^2 peaks there.  Catches sign, orientation, shift, scale."""
    N, A, T, s = 32, 24, 3, 3 + 1j
    xy, f, g, ef = _on_cell_plane_wave(A, ql, qm, s, T)
    img = oracle.image(xy, f, g, ef, N)[0, 0].real
    k = np.arange(N) - N // 2                                    # shifted pixel order
    b1 = 1 + 2 * E2 * np.cos(2 * np.pi * k / N)
    B2 = np.outer(b1, b1) ** 2
    row, col = qm + N // 2, ql + N // 2
    expect = T * abs(s) ** 2 * A ** 2 * B2[row, col]
    assert abs(img[row, col] - expect) / expect < 1e-12
    q = np.unravel_index(np.argmax(img / B2), img.shape)
    assert q == (row, col)


def test_p2_zenith_closed_form_off_cell():
    """Zenith source on arbitrary (off-cell) antennas: every antenna sees the same
    integer sample s, so XX(zenith) = T |s|^2 |sum_a g_a sum_taps w_a|^2."""
    rng = _rng(7)
    A, N, T = 10, 32, 4
    xy = rng.uniform(-9, 9, size=(A, 2))
    f = np.array([50e6])
    g = synth.random_gains(rng, (1, 1, A))
    s = -5 + 2j
    ef = np.full((T, 1, 1, A), synth.pack_ci4(np.array(s.real), np.array(s.imag)), np.uint8)
    img = oracle.image(xy, f, g, ef, N)[0, 0]
    cell = oracle.C0 / 50e6 * 0.5
    X = xy[:, 0] / cell + N / 2
    Y = xy[:, 1] / cell + N / 2
    wsum = np.zeros(A)
    for a in range(A):                       # the Gaussian's definition, per tap
        i0, j0 = np.floor(X[a] + 0.5), np.floor(Y[a] + 0.5)
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                wsum[a] += np.exp(-2.0 * ((i0 + di - X[a]) ** 2 + (j0 + dj - Y[a]) ** 2))
    expect = T * abs(s) ** 2 * abs(np.sum(g[0, 0].astype(complex) * wsum)) ** 2
    assert abs(img[N // 2, N // 2].real - expect) / expect < 1e-12
    assert abs(img[N // 2, N // 2].imag) < 1e-9 * expect


# ------------------------------------------------------------------ P3
def test_p3_parseval():
    inp = synth.random_problem(11, 32, 12, 2, 2, 5, fill=0.4)
    img = oracle.image_from(inp)
    X, Y = oracle.antenna_cells(inp.xy_m, inp.freq_hz, 32)
    ii, jj, w = oracle.kernel_taps(X, Y, 32)
    e = oracle.unpack_ci4(inp.efield)
    ng = 32 * 32
    for c in range(2):
        A = oracle.grid_efield(inp.gains[c].astype(complex)[None] * e[:, c], ii[c], jj[c], w[c], 32)
        ax, ay = A[:, 0], A[:, 1]
        pxx = ng * np.sum(np.abs(ax) ** 2)
        pyy = ng * np.sum(np.abs(ay) ** 2)
        pxy = ng * np.sum(ax * np.conj(ay))
        assert abs(img[c, 0].sum() - pxx) / pxx < 1e-12
        assert abs(img[c, 3].sum() - pyy) / pyy < 1e-12
        assert abs(img[c, 1].sum() - pxy) / abs(pxy) < 1e-11
        assert abs(img[c, 2].sum() - np.conj(pxy)) / abs(pxy) < 1e-11


# ------------------------------------------------------------------ P4
def test_p4_autocorrelation_identity():
    """I_PQ(k) = sum_delta C_PQ(delta) e^{+2 pi i delta k / N}, C the circular
    correlation of the gridded fields summed over time, by direct sums."""
    N = 16
    inp = synth.random_problem(12, N, 6, 1, 2, 3, fill=0.45)
    img = np.fft.ifftshift(oracle.image_from(inp)[0], axes=(-2, -1))
    X, Y = oracle.antenna_cells(inp.xy_m, inp.freq_hz, N)
    ii, jj, w = oracle.kernel_taps(X, Y, N)
    e = oracle.unpack_ci4(inp.efield)
    A = oracle.grid_efield(inp.gains[0].astype(complex)[None] * e[:, 0], ii[0], jj[0], w[0], N)
    pairs = [(0, 0), (0, 1), (1, 0), (1, 1)]
    for n, (p, q) in enumerate(pairs):
        C = np.zeros((N, N), complex)
        for dy in range(N):
            for dx in range(N):
                shifted = np.roll(A[:, p], shift=(-dy, -dx), axis=(-2, -1))   # A_P(h + delta)
                C[dy, dx] = np.sum(shifted * np.conj(A[:, q]))
        I = oracle.direct_dft(C)
        assert np.linalg.norm(I - img[n]) / np.linalg.norm(img[n]) < 1e-11


# ------------------------------------------------------------------ P5
@pytest.mark.parametrize("seed,N,A,C,P,T", [(21, 32, 16, 2, 2, 6), (22, 32, 9, 1, 1, 4),
                                          (23, 16, 5, 3, 2, 2)])
def test_p5_fx_form_equals_moff(seed, N, A, C, P, T):
    """The MOFF image equals the visibility-based image (paper §2, Eq. (1) <-> (5))."""
    inp = synth.random_problem(seed, N, A, C, P, T, fill=0.45)
    img = oracle.image_from(inp)
    fx = oracle.image_fx(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, N)
    assert np.linalg.norm(fx - img) / np.linalg.norm(img) < 1e-11


# ------------------------------------------------------------------ P6
def test_p6_linearity_and_single_antenna():
    inp = synth.random_problem(31, 32, 8, 1, 2, 4)
    img = oracle.image_from(inp)
    s = 0.7 - 1.3j
    img_s = oracle.image(inp.xy_m, inp.freq_hz, inp.gains.astype(complex) * s,
                         inp.efield, 32)
    assert np.allclose(img_s, abs(s) ** 2 * img, rtol=1e-13, atol=1e-9)
    zero = np.zeros_like(inp.efield)
    assert np.all(oracle.image(inp.xy_m, inp.freq_hz, inp.gains, zero, 32) == 0)
    # single antenna: XX = sum_t |g e_t|^2 |B_a(k)|^2, B_a separable per axis
    one = synth.random_problem(32, 32, 1, 1, 1, 3)
    img1 = np.fft.ifftshift(oracle.image_from(one)[0, 0], axes=(-2, -1)).real
    cell = oracle.C0 / one.freq_hz[0] * 0.5
    X = one.xy_m[0, 0] / cell + 16
    Y = one.xy_m[0, 1] / cell + 16
    k = np.arange(32)

    def axis_resp(x):
        i0 = np.floor(x + 0.5)
        return sum(np.exp(-2.0 * (i0 + d - x) ** 2) * np.exp(2j * np.pi * (i0 + d) * k / 32)
                   for d in (-1, 0, 1))
    e = oracle.unpack_ci4(one.efield[:, 0, 0, 0]) * complex(one.gains[0, 0, 0])
    expect = np.sum(np.abs(e) ** 2) * np.outer(np.abs(axis_resp(Y)) ** 2, np.abs(axis_resp(X)) ** 2)
    assert np.allclose(img1, expect, rtol=1e-12, atol=1e-12 * expect.max())


# ------------------------------------------------------------------ P7, P9
def test_p7_p9_symmetries_and_cauchy_schwarz():
    inp = synth.random_problem(41, 32, 10, 2, 2, 5)
    img = oracle.image_from(inp)
    xx, xy, yx, yy = img[:, 0], img[:, 1], img[:, 2], img[:, 3]
    assert np.all(xx.imag == 0) and np.all(yy.imag == 0)
    assert np.all(xx.real >= 0) and np.all(yy.real >= 0)
    assert np.array_equal(yx, np.conj(xy))
    assert np.all(np.abs(xy) ** 2 <= xx.real * yy.real * (1 + 1e-12) + 1e-9)


# ------------------------------------------------------------------ P8
def test_p8_whole_cell_translation_invariance():
    inp = synth.random_problem(51, 32, 10, 1, 2, 4, fill=0.35)
    img = oracle.image_from(inp)
    cell = oracle.C0 / inp.freq_hz[0] * 0.5
    moved = inp.xy_m + np.array([3 * cell, -2 * cell])
    img2 = oracle.image(moved, inp.freq_hz, inp.gains, inp.efield, 32)
    assert np.linalg.norm(img2 - img) / np.linalg.norm(img) < 1e-12


# ------------------------------------------------------------------ P12
def test_p12_time_splitting():
    inp = synth.random_problem(61, 32, 8, 2, 2, 9)
    full = oracle.image_from(inp)
    a = oracle.image(inp.xy_m, inp.freq_hz, inp.gains, inp.efield[:4], 32)
    b = oracle.image(inp.xy_m, inp.freq_hz, inp.gains, inp.efield[4:], 32)
    assert np.linalg.norm(a + b - full) / np.linalg.norm(full) < 1e-14


# ------------------------------------------------------------------ P10, P11
def _loss_setup(seed, N=32, A=8, C=2, P=2, T=3):
    inp = synth.random_problem(seed, N, A, C, P, T, fill=0.4)
    model = oracle.image_from(inp) * 0.0
    rng = _rng(seed + 100)
    model = model + rng.normal(size=model.shape) * 50.0      # any fixed M
    g = inp.gains.astype(np.complex128)

    def loss(gg):
        return oracle.l2_loss(oracle.image(inp.xy_m, inp.freq_hz, gg, inp.efield, N), model)
    return inp, model, g, loss


@pytest.mark.parametrize("P", [1, 2])
def test_p10_gradient_matches_finite_differences(P):
    inp, model, g, loss = _loss_setup(71 + P, P=P, A=6 if P == 2 else 8)
    img = oracle.image(inp.xy_m, inp.freq_hz, g, inp.efield, 32)
    gam = oracle.l2_loss_grad_image(img, model)
    grad = oracle.grad_gains(inp.xy_m, inp.freq_hz, g, inp.efield, 32, gam)
    coords = [tuple(i) for i in np.ndindex(*g.shape)]
    fd = oracle.fd_grad(loss, g, coords)
    an = np.array([grad[c] for c in coords])
    assert np.linalg.norm(an - fd) / np.linalg.norm(fd) < 1e-6


def test_p10_gradient_of_cross_products_only():
    """A loss on XY alone (XX, YY excluded) checks the h-terms of the chain."""
    inp = synth.random_problem(81, 32, 5, 1, 2, 3, fill=0.4)
    g = inp.gains.astype(np.complex128)
    rng = _rng(5)
    wxy = rng.normal(size=(1, 32, 32)) + 1j * rng.normal(size=(1, 32, 32))

    def loss(gg):
        im = oracle.image(inp.xy_m, inp.freq_hz, gg, inp.efield, 32)
        return float(np.sum((np.conj(wxy) * im[:, 1]).real))
    gam = np.zeros((1, 4, 32, 32), complex)
    gam[:, 1] = wxy                     # dL/dRe(XY) + i dL/dIm(XY)
    grad = oracle.grad_gains(inp.xy_m, inp.freq_hz, g, inp.efield, 32, gam)
    coords = [tuple(i) for i in np.ndindex(*g.shape)]
    fd = oracle.fd_grad(loss, g, coords)
    an = np.array([grad[c] for c in coords])
    assert np.linalg.norm(an - fd) / np.linalg.norm(fd) < 1e-6


def test_p11_gradient_invariants():
    inp, model, g, loss = _loss_setup(91, A=10)
    img = oracle.image(inp.xy_m, inp.freq_hz, g, inp.efield, 32)
    gam = oracle.l2_loss_grad_image(img, model)
    grad = oracle.grad_gains(inp.xy_m, inp.freq_hz, g, inp.efield, 32, gam)
    # (i) a common phase per channel leaves every product unchanged
    for c in range(g.shape[0]):
        s = np.sum(np.conj(g[c]) * grad[c])
        assert abs(s.imag) < 1e-10 * np.sum(np.abs(g[c] * grad[c]))
    # (ii) degree-2 homogeneity: Re sum conj(g) grad = 2 sum Re(conj(Gamma) I)
    lhs = np.sum(np.conj(g) * grad).real
    rhs = 2.0 * np.sum((np.conj(gam) * img).real)
    assert abs(lhs - rhs) / abs(rhs) < 1e-12


# ------------------------------------------------------------------ generator
def test_config2_generator_statistics():
    inp = synth.config2(n_time=40, n_chan=3)
    e = oracle.unpack_ci4(inp.efield)
    clipped = np.mean((e.real == -8) | (e.real == 7) | (e.imag == -8) | (e.imag == 7))
    assert clipped < 0.005
    d = np.sqrt(((inp.xy_m[:, None] - inp.xy_m[None]) ** 2).sum(-1)) + np.eye(256) * 1e9
    assert d.min() >= 4.5 - 1e-9
    assert np.all(np.hypot(inp.xy_m[:, 0], inp.xy_m[:, 1]) <= 50.0)
    oracle.kernel_taps(*oracle.antenna_cells(inp.xy_m, inp.freq_hz, 64), 64)   # on grid


def test_cost_model_grid_scaling():
    """n_g log2 n_g predicts x4.7 from 64^2 to 128^2 (paper §5.1)."""
    r = (128 ** 2 * np.log2(128 ** 2)) / (64 ** 2 * np.log2(64 ** 2))
    assert abs(r - 4.67) < 0.01


# ------------------------------------------------ autocorrelation removal
def _small(seed, N=32, A=12, C=2, P=2, T=5):
    return synth.random_problem(seed, N, A, C, P, T)


def test_p13_autos_removed_equals_fx_form_without_diagonal():
    """Image (gridding + FFT path) minus the autocorrelation image equals the
    visibility form with the a = b entries removed (an independent route)."""
    inp = _small(501)
    got = oracle.image_without_autos_from(inp)
    V = oracle.visibilities(inp.gains, inp.efield)
    A = inp.n_ant
    V[:, :, np.arange(A), np.arange(A)] = 0.0
    ref = oracle.image_fx(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, inp.grid_n, vis=V)
    scale = np.abs(oracle.image_from(inp)).max()
    assert np.max(np.abs(got - ref)) <= 1e-11 * scale


def test_p13_single_antenna_leaves_nothing():
    inp = _small(502, A=1)
    full = oracle.image_from(inp)
    got = oracle.image_without_autos_from(inp)
    assert np.max(np.abs(got)) <= 1e-12 * np.abs(full).max()


def test_p13_zenith_autocorrelation_closed_form():
    """At the zenith pixel |b_a(0)|^2 = (sum of the antenna's tap weights)^2."""
    inp = _small(503, P=1)
    N = inp.grid_n
    auto = oracle.autocorrelation_image(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, N)
    X, Y = oracle.antenna_cells(inp.xy_m, inp.freq_hz, N)
    _, _, w = oracle.kernel_taps(X, Y, N)
    e = oracle.unpack_ci4(inp.efield)[:, :, 0]                        # [T, C, A]
    g = inp.gains[:, 0].astype(np.complex128)                         # [C, A]
    for c in range(inp.n_chan):
        power = np.sum(np.abs(g[c][None] * e[:, c]) ** 2, axis=0)    # [A]
        ref = np.sum(power * w[c].sum(axis=1) ** 2)
        assert abs(auto[c, 0, N // 2, N // 2] - ref) <= 1e-12 * ref


def test_p13_autocorrelations_split_over_time_and_conjugate():
    inp = _small(504, T=7)
    a = oracle.autocorrelation_image(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, inp.grid_n)
    a1 = oracle.autocorrelation_image(inp.xy_m, inp.freq_hz, inp.gains, inp.efield[:3], inp.grid_n)
    a2 = oracle.autocorrelation_image(inp.xy_m, inp.freq_hz, inp.gains, inp.efield[3:], inp.grid_n)
    assert np.max(np.abs(a - a1 - a2)) <= 1e-12 * np.abs(a).max()
    assert np.max(np.abs(a[:, 2] - np.conj(a[:, 1]))) <= 1e-12 * np.abs(a).max()
    assert np.all(a[:, 0].real >= 0) and np.max(np.abs(a[:, 0].imag)) <= 1e-12 * np.abs(a).max()


# ------------------------------------------------ P14: gradient without autos
def _loss_without_autos(inp, model):
    def loss(gg):
        return oracle.l2_loss(oracle.image_without_autos(inp.xy_m, inp.freq_hz, gg, inp.efield,
                                                         inp.grid_n), model)
    return loss


@pytest.mark.parametrize("P", [1, 2])
def test_p14_gradient_without_autos_matches_finite_differences(P):
    """Gradient of a loss on the image with the autocorrelations removed
    (Sec. 3.2) against central differences of that loss."""
    inp, model, g, _ = _loss_setup(171 + P, P=P, A=6 if P == 2 else 8)
    img = oracle.image_without_autos(inp.xy_m, inp.freq_hz, g, inp.efield, 32)
    gam = oracle.l2_loss_grad_image(img, model)
    grad = oracle.grad_gains_without_autos(inp.xy_m, inp.freq_hz, g, inp.efield, 32, gam)
    coords = [tuple(i) for i in np.ndindex(*g.shape)]
    fd = oracle.fd_grad(_loss_without_autos(inp, model), g, coords)
    an = np.array([grad[c] for c in coords])
    assert np.linalg.norm(an - fd) / np.linalg.norm(fd) < 1e-6


def test_p14_gradient_without_autos_cross_products_only():
    """A loss on XY and YX alone checks the cross-polarisation terms."""
    inp = synth.random_problem(181, 32, 5, 1, 2, 3, fill=0.4)
    g = inp.gains.astype(np.complex128)
    rng = _rng(6)
    wxy = rng.normal(size=(1, 32, 32)) + 1j * rng.normal(size=(1, 32, 32))
    wyx = rng.normal(size=(1, 32, 32)) + 1j * rng.normal(size=(1, 32, 32))

    def loss(gg):
        im = oracle.image_without_autos(inp.xy_m, inp.freq_hz, gg, inp.efield, 32)
        return float(np.sum((np.conj(wxy) * im[:, 1]).real + (np.conj(wyx) * im[:, 2]).real))
    gam = np.zeros((1, 4, 32, 32), complex)
    gam[:, 1], gam[:, 2] = wxy, wyx
    grad = oracle.grad_gains_without_autos(inp.xy_m, inp.freq_hz, g, inp.efield, 32, gam)
    coords = [tuple(i) for i in np.ndindex(*g.shape)]
    fd = oracle.fd_grad(loss, g, coords)
    an = np.array([grad[c] for c in coords])
    assert np.linalg.norm(an - fd) / np.linalg.norm(fd) < 1e-6


def test_p14_single_antenna_gradient_vanishes():
    """One antenna: the image without autocorrelations is zero for every gain,
    so its gradient is zero whatever the upstream gradient."""
    inp = synth.random_problem(182, 32, 1, 2, 2, 4)
    rng = _rng(7)
    gam = rng.normal(size=(2, 4, 32, 32)) + 1j * rng.normal(size=(2, 4, 32, 32))
    full = oracle.grad_gains(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 32, gam)
    grad = oracle.grad_gains_without_autos(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 32, gam)
    assert np.max(np.abs(grad)) <= 1e-12 * np.max(np.abs(full))


def test_p14_homogeneity_without_autos():
    """Degree-2 homogeneity in the gains holds for the removed image too."""
    inp, model, g, _ = _loss_setup(191, A=10)
    img = oracle.image_without_autos(inp.xy_m, inp.freq_hz, g, inp.efield, 32)
    gam = oracle.l2_loss_grad_image(img, model)
    grad = oracle.grad_gains_without_autos(inp.xy_m, inp.freq_hz, g, inp.efield, 32, gam)
    lhs = np.sum(np.conj(g) * grad).real
    rhs = 2.0 * np.sum((np.conj(gam) * img).real)
    assert abs(lhs - rhs) / abs(rhs) < 1e-12


# ------------------------------------------------------- P15: front end (§3.2)
@pytest.mark.parametrize("c0,c_step,n_chan", [(0, 1, 5), (2, 1, 3), (1, 2, 3), (4, 3, 1), (0, 5, 2)])
@pytest.mark.parametrize("P", [1, 2])
def test_p15_decimate_transpose_by_loops(c0, c_step, n_chan, P):
    """Decimation and transposition against explicit loops over every byte."""
    raw = synth.raw_gulp(7, 3, 9, 5, P)
    got = oracle.decimate_transpose(raw, n_chan, c0, c_step)
    T, c_in, A, _ = raw.shape
    assert got.shape == (T, n_chan, P, A)
    for t in range(T):
        for i in range(n_chan):
            for p in range(P):
                for a in range(A):
                    assert got[t, i, p, a] == raw[t, c0 + i * c_step, a, p]


def test_p15_front_end_rejects_selections_outside_the_input():
    raw = synth.raw_gulp(8, 2, 6, 3, 2)
    for c0, c_step, n in [(-1, 1, 2), (0, 0, 2), (5, 1, 2), (0, 3, 3), (0, 1, 0)]:
        with pytest.raises(ValueError):
            oracle.decimate_transpose(raw, n, c0, c_step)


def test_p15_front_end_then_image_equals_image_of_the_selected_data():
    """The image of a decimated, transposed gulp equals the image of the same
    channels' data given directly in [T, C, P, A] order (built here by loops)."""
    inp = synth.random_problem(151, 32, 12, 3, 2, 4)
    c_in, c0, step = 8, 1, 3
    raw = synth.raw_gulp(152, 4, c_in, 12, 2)
    direct = np.empty((4, 3, 2, 12), np.uint8)
    for t in range(4):
        for i in range(3):
            for p in range(2):
                for a in range(12):
                    direct[t, i, p, a] = raw[t, c0 + i * step, a, p]
    ef = oracle.decimate_transpose(raw, 3, c0, step)
    a = oracle.image(inp.xy_m, inp.freq_hz, inp.gains, ef, 32)
    b = oracle.image(inp.xy_m, inp.freq_hz, inp.gains, direct, 32)
    assert np.array_equal(a, b)


# ------------------------------------------- P16: user (complex) kernels (§3.3)
def _kinp(seed, K, A=9, C=2, P=2, T=3, N=32, fill=0.3):
    return synth.with_kernels(synth.random_problem(seed, N, A, C, P, T, fill=fill), K, seed + 1)


@pytest.mark.parametrize("K", [3, 5, 9])
def test_p16_fx_form_with_complex_kernels(K):
    """The visibility form with each antenna's own complex kernel equals the
    MOFF image gridded with those kernels (§2.1 Eq. (1) <-> Eq. (5))."""
    inp = _kinp(160 + K, K)
    a = oracle.image_from(inp)
    b = oracle.image_fx(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 32, K, 0.5, 0.5,
                        kernels=inp.kernels)
    assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(a))


def test_p16_kernel_phase_moves_into_the_gain():
    """A kernel multiplies the calibrated sample like a gain does: a unit phase
    per antenna taken off the gains and put on the kernels leaves every product
    unchanged (catches a conjugated kernel in the gridding)."""
    inp = _kinp(170, 5)
    phase = np.exp(1j * np.random.default_rng(171).uniform(0, 2 * np.pi, size=(2, 1, 9)))
    g2 = inp.gains.astype(complex) * phase
    k2 = inp.kernels.astype(complex) * np.conj(phase[:, 0, :, None, None])
    a = oracle.image_from(inp)
    b = oracle.image(inp.xy_m, inp.freq_hz, g2, inp.efield, 32, 5, 0.5, 0.5, kernels=k2)
    assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(a))


def test_p16_single_antenna_closed_form_complex_kernel():
    """One antenna: XX(k) = sum_t |g e_t|^2 |sum_taps w e^{+2 pi i (i kl + j km)/N}|^2,
    the kernel's own transform evaluated here by a direct sum over its taps."""
    inp = _kinp(180, 7, A=1, C=1, P=1, T=5)
    N, K, h = 32, 7, 3
    got = np.fft.ifftshift(oracle.image_from(inp)[0, 0], axes=(-2, -1)).real
    X, Y = oracle.antenna_cells(inp.xy_m, inp.freq_hz, N)
    i0, j0 = int(np.floor(X[0, 0] + 0.5)), int(np.floor(Y[0, 0] + 0.5))
    k = np.arange(N)
    b = np.zeros((N, N), complex)
    for dj in range(-h, h + 1):
        for di in range(-h, h + 1):
            w = complex(inp.kernels[0, 0, dj + h, di + h])
            b += w * np.exp(2j * np.pi * ((j0 + dj) * k[:, None] + (i0 + di) * k[None, :]) / N)
    e = oracle.unpack_ci4(inp.efield[:, 0, 0, 0])
    power = np.sum(np.abs(complex(inp.gains[0, 0, 0]) * e) ** 2)
    assert np.max(np.abs(got - power * np.abs(b) ** 2)) <= 1e-11 * np.max(got)


@pytest.mark.parametrize("P", [1, 2])
def test_p16_gradient_with_complex_kernels_matches_finite_differences(P):
    inp = _kinp(190 + P, 5, A=6, P=P)
    rng = _rng(192)
    model = rng.normal(size=oracle.image_from(inp).shape) * 50.0
    g = inp.gains.astype(np.complex128)

    def loss(gg):
        return oracle.l2_loss(oracle.image(inp.xy_m, inp.freq_hz, gg, inp.efield, 32, 5,
                                           kernels=inp.kernels), model)
    img = oracle.image(inp.xy_m, inp.freq_hz, g, inp.efield, 32, 5, kernels=inp.kernels)
    gam = oracle.l2_loss_grad_image(img, model)
    grad = oracle.grad_gains(inp.xy_m, inp.freq_hz, g, inp.efield, 32, gam, 5,
                             kernels=inp.kernels)
    coords = [tuple(i) for i in np.ndindex(*g.shape)]
    fd = oracle.fd_grad(loss, g, coords)
    an = np.array([grad[c] for c in coords])
    assert np.linalg.norm(an - fd) / np.linalg.norm(fd) < 1e-6


def test_p16_kernels_shape_checked():
    inp = _kinp(195, 3)
    with pytest.raises(ValueError):
        oracle.image(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 32, 5, kernels=inp.kernels)


# ------------------------------------------------- P17: post-processing (§3.2, §4.3)
def _one_antenna_pol(ex, ey, T=6, N=32):
    """One antenna, unit gain, every sample E_X = ex, E_Y = ey (int4 complex)."""
    inp = synth.random_problem(200, N, 1, 1, 2, T)
    byte = lambda z: ((int(z.real) & 0xF) << 4) | (int(z.imag) & 0xF)
    ef = np.empty((T, 1, 2, 1), np.uint8)
    ef[:, 0, 0, 0] = byte(ex)
    ef[:, 0, 1, 0] = byte(ey)
    gains = np.ones((1, 2, 1), np.complex64)
    return oracle.image(inp.xy_m, inp.freq_hz, gains, ef, N)


@pytest.mark.parametrize("ex,ey,q,u,v", [(4, 0, 1, 0, 0), (0, 4, -1, 0, 0), (3, 3, 0, 1, 0),
                                         (3, -3, 0, -1, 0), (4, 4j, 0, 0, -1), (4, -4j, 0, 0, 1)])
def test_p17_pseudo_stokes_of_pure_polarisation_states(ex, ey, q, u, v):
    """Textbook states: X only (Q = I), Y only (Q = -I), +-45 deg linear (U = +-I),
    E_Y = +-i E_X (V = -+I), at every pixel of a one-antenna image."""
    st = oracle.pseudo_stokes(_one_antenna_pol(complex(ex), complex(ey)))
    I = st[0, 0]
    assert np.all(I > 0)
    for plane, want in ((1, q), (2, u), (3, v)):
        assert np.max(np.abs(st[0, plane] - want * I)) <= 1e-12 * I.max()


def test_p17_taper_correction_is_exact_for_identical_kernels():
    """Antennas on whole cells all have the same Gaussian kernel, so each product
    is the point-kernel image times T = |kernel transform|^2: dividing by
    kernel_taper recovers the image gridded with a unit 1 x 1 kernel."""
    N, A, T = 32, 7, 4
    inp = synth.random_problem(201, N, A, 1, 2, T)
    cell_m = oracle.C0 / inp.freq_hz[0] * 0.5
    rng = np.random.default_rng(202)
    cells = rng.choice(np.arange(-6, 7), size=(A, 2))
    xy = cells * cell_m
    img = oracle.image(xy, inp.freq_hz, inp.gains, inp.efield, N, 3, 0.5)
    ones = np.ones((1, A, 1, 1), complex)
    point = oracle.image(xy, inp.freq_hz, inp.gains, inp.efield, N, 1, 0.5, kernels=ones)
    taper = oracle.kernel_taper(xy, inp.freq_hz, N, 3, 0.5)
    floor = 1e-3
    got = oracle.taper_corrected(oracle.pseudo_stokes(img), taper, floor)
    want = oracle.pseudo_stokes(point)
    keep = taper[0] >= floor * taper.max()
    assert keep.sum() > N * N // 2
    assert np.max(np.abs(got[0][:, keep] - want[0][:, keep])) <= 1e-9 * np.abs(want).max()
    assert np.all(got[0][:, ~keep] == 0)


def test_p17_taper_of_a_unit_point_kernel_is_one():
    inp = synth.random_problem(203, 32, 5, 2, 1, 1)
    ones = np.ones((2, 5, 1, 1), complex)
    t = oracle.kernel_taper(inp.xy_m, inp.freq_hz, 32, 1, 0.5, kernels=ones)
    assert np.max(np.abs(t - 1.0)) <= 1e-12


def test_p16_autos_removed_with_complex_kernels_equals_fx_form_without_diagonal():
    """With each antenna's own complex kernel, the image minus its
    autocorrelation image is still the visibility form without its diagonal."""
    inp = _kinp(230, 5, A=8, C=2, P=2, T=4)
    got = oracle.image_without_autos_from(inp)
    V = oracle.visibilities(inp.gains, inp.efield)
    V[:, :, np.arange(8), np.arange(8)] = 0.0
    ref = oracle.image_fx(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 32, 5, 0.5, 0.5, vis=V,
                          kernels=inp.kernels)
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.abs(oracle.image_from(inp)).max()


def test_p16_gradient_without_autos_with_complex_kernels_matches_finite_differences():
    inp = _kinp(231, 3, A=6, C=1, P=2, T=3)
    rng = _rng(232)
    model = rng.normal(size=oracle.image_from(inp).shape) * 20.0
    g = inp.gains.astype(np.complex128)

    def loss(gg):
        return oracle.l2_loss(oracle.image_without_autos(inp.xy_m, inp.freq_hz, gg, inp.efield, 32,
                                                         3, kernels=inp.kernels), model)
    img = oracle.image_without_autos(inp.xy_m, inp.freq_hz, g, inp.efield, 32, 3,
                                     kernels=inp.kernels)
    gam = oracle.l2_loss_grad_image(img, model)
    grad = oracle.grad_gains_without_autos(inp.xy_m, inp.freq_hz, g, inp.efield, 32, gam, 3,
                                           kernels=inp.kernels)
    coords = [tuple(i) for i in np.ndindex(*g.shape)]
    fd = oracle.fd_grad(loss, g, coords)
    an = np.array([grad[c] for c in coords])
    assert np.linalg.norm(an - fd) / np.linalg.norm(fd) < 1e-6


# ------------------------------------------------------------------ P18 (O11)
def _whole_cell_array(n_ant, seed, N=32, freq=50e6):
    """Antennas on distinct whole cells within +-8 cells of the centre."""
    rng = _rng(seed)
    cells = set()
    while len(cells) < n_ant:
        cells.add(tuple(int(v) for v in rng.integers(-8, 9, size=2)))
    cxy = np.array(sorted(cells), dtype=float)
    return cxy, cxy * (oracle.C0 / freq * 0.5), np.array([freq])


@pytest.mark.parametrize("n_pol", [1, 2])
def test_p18_model_image_whole_cell_closed_form(n_pol):
    """Model image of point sources on whole-cell antennas, every pixel.

    Antenna a at relative cell (cx, cy) has the footprint transform
    b_a(k) = e^{2 pi i ((cx + N/2) kl + (cy + N/2) km)/N} B(k), with the hand
    Gaussian B(k) = (1 + 2e^-2 cos(2 pi kl/N))(1 + 2e^-2 cos(2 pi km/N)).  A
    source at the on-pixel direction (ql, qm) (l = ql / (N du)) reaches it with
    phase e^{-2 pi i (cx ql + cy qm)/N}, so the model visibilities
    V = T (sum_s S_s p_s p_s^H + 2 sigma^2 Id) image to
        XX(k) = YY(k) = T B(k)^2 [ sum_s S_s |AF_s(k)|^2 + 2 sigma^2 A ],
    AF_s(k) = sum_a e^{2 pi i (cx (kl - ql_s) + cy (km - qm_s))/N} (array factor,
    summed here antenna by antenna), and XY = YX = 0.  Catches the sign of the
    source phase (sources mirrored), a missing T, the noise term's factor,
    |.| not squared and the pixel order."""
    N, A, T, sigma = 32, 14, 7, 1.5
    cxy, xy, f = _whole_cell_array(A, 3)
    q = [(5, -3), (-9, 2), (0, 11)]
    S = [2.0, 0.7, 1.3]
    lm = np.array([[ql / (N * 0.5), qm / (N * 0.5)] for ql, qm in q])
    got = oracle.model_image(xy, f, N, T, lm, np.array(S), sigma, n_pol=n_pol)
    k = np.arange(N) - N // 2                       # shifted pixel order
    b1 = 1 + 2 * E2 * np.cos(2 * np.pi * k / N)
    B2 = np.outer(b1, b1) ** 2                      # [row km, col kl]
    km, kl = np.meshgrid(k, k, indexing="ij")
    expect = np.full((N, N), 2 * sigma ** 2 * A)
    for (ql, qm), s in zip(q, S):
        af = np.zeros((N, N), complex)
        for cx, cy in cxy:
            af += np.exp(2j * np.pi * (cx * (kl - ql) + cy * (km - qm)) / N)
        expect += s * np.abs(af) ** 2
    expect *= T * B2
    assert got.shape == (1, 1 if n_pol == 1 else 4, N, N)
    assert np.max(np.abs(got[0, 0] - expect)) <= 1e-12 * expect.max()
    if n_pol == 2:
        assert np.max(np.abs(got[0, 3] - expect)) <= 1e-12 * expect.max()
        assert np.all(got[0, 1] == 0) and np.all(got[0, 2] == 0)
    # each source's own pixel holds T B^2 (S A^2 + the others' sidelobes + noise)
    r, c = q[0][1] + N // 2, q[0][0] + N // 2
    assert got[0, 0, r, c].real >= T * B2[r, c] * S[0] * A ** 2


def test_p18_model_image_zenith_off_cell():
    """Off-cell antennas, zenith pixel: a source at the zenith adds
    T S (sum_a sum_taps w_a)^2 and the noise term is 2 sigma^2 T sum_a (sum_taps w_a)^2,
    with w the Gaussian evaluated tap by tap from its definition."""
    rng = _rng(17)
    A, N, T, sigma, S = 11, 32, 5, 2.0, 3.5
    xy = rng.uniform(-9, 9, size=(A, 2))
    f = np.array([50e6])
    cell = oracle.C0 / 50e6 * 0.5
    X = xy[:, 0] / cell + N / 2
    Y = xy[:, 1] / cell + N / 2
    wsum = np.zeros(A)
    for a in range(A):
        i0, j0 = np.floor(X[a] + 0.5), np.floor(Y[a] + 0.5)
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                wsum[a] += np.exp(-2.0 * ((i0 + di - X[a]) ** 2 + (j0 + dj - Y[a]) ** 2))
    noise_only = oracle.model_image(xy, f, N, T, np.zeros((0, 2)), np.zeros(0), sigma)
    expect_n = 2 * sigma ** 2 * T * np.sum(wsum ** 2)
    assert abs(noise_only[0, 0, N // 2, N // 2].real - expect_n) <= 1e-12 * expect_n
    both = oracle.model_image(xy, f, N, T, np.zeros((1, 2)), np.array([S]), sigma)
    expect = expect_n + T * S * np.sum(wsum) ** 2
    assert abs(both[0, 3, N // 2, N // 2].real - expect) <= 1e-12 * expect


def test_p18_model_image_is_the_mean_of_simulated_images():
    """The model is what the imager sees on average: the oracle image of data
    drawn from the same sky (unit gains, a source 4x brighter than the noise
    in the image, no clipping) matches the model within the sampling error of
    4000 samples once the int4 rounding (uniform, variance 1/12 per
    component) is added to the noise power; a model with the source mirrored
    or the noise power halved is 25x further off."""
    N, A, T = 32, 10, 4000
    cxy, xy, f = _whole_cell_array(A, 9)
    sigma = 1.5
    lm = np.array([[4 / 16, -2 / 16]])
    power = np.array([2.0])
    ef = synth.simulate_efield(_rng(31), _rng(32), xy, f, T, 1, lm, np.sqrt(power),
                               np.zeros(1), sigma)
    got = oracle.image(xy, f, np.ones((1, 1, A), np.complex64), ef, N)
    s_eff = np.sqrt(sigma ** 2 + 1 / 12)

    def err(m):
        return np.linalg.norm(got - m) / np.linalg.norm(m)
    assert err(oracle.model_image(xy, f, N, T, lm, power, s_eff, n_pol=1)) < 0.03
    assert err(oracle.model_image(xy, f, N, T, -lm, power, s_eff, n_pol=1)) > 0.3
    assert err(oracle.model_image(xy, f, N, T, lm, power, s_eff / np.sqrt(2), n_pol=1)) > 0.3


# ------------------------------------------------------------------ P19 (Q27)
def test_p19_error_metric_hand_values():
    """rel_errors on hand-built 2 x 2 images with known norms: XX, YY relative to
    their own norms; XY, YX relative to sqrt(||XX|| ||YY||)."""
    ref = np.zeros((2, 4, 2, 2), complex)
    ref[0, 0] = [[3, 0], [0, 4]]                 # ||XX|| = 5
    ref[0, 3] = [[0, 0], [0, 20]]                # ||YY|| = 20 -> scale 10
    ref[0, 1] = [[1j, 0], [0, 0]]                # ||XY|| = 1 (not the scale)
    ref[0, 2] = np.conj(ref[0, 1])
    ref[1, 0] = [[0, 0], [6, 8]]                 # ||XX|| = 10
    ref[1, 3] = [[0, 2.5], [0, 0]]               # ||YY|| = 2.5 -> scale 5
    img = ref.copy()
    img[0, 0, 0, 1] += 0.3 + 0.4j                # |d| = 0.5 -> 0.1
    img[0, 3, 1, 0] -= 2.0                       # 2 / 20 = 0.1
    img[0, 1, 1, 1] += 0.5                       # 0.5 / 10 = 0.05
    img[0, 2, 0, 0] += 3.0                       # 3 / 10 = 0.3
    img[1, 0] += 1.0                             # ||d|| = 2 -> 0.2
    img[1, 1, 0, 0] += 1.2 - 1.6j                # 2 / 5 = 0.4
    img[1, 2, 1, 1] += 0.05                      # 0.05 / 5 = 0.01
    img[1, 3, 0, 1] += 0.25                      # 0.25 / 2.5 = 0.1
    got = oracle.rel_errors(img, ref)
    expect = np.array([[0.1, 0.05, 0.3, 0.1], [0.2, 0.4, 0.01, 0.1]])
    assert np.allclose(got, expect, rtol=1e-14, atol=0)
    one = oracle.rel_errors(img[:, :1], ref[:, :1])
    assert np.allclose(one[:, 0], [0.1, 0.2], rtol=1e-14, atol=0)


# ------------------------------------------------------------------ P10 at the calibration shape
@pytest.mark.slow
def test_p10_calibration_shape_finite_differences():
    """The calibration workload at its full shape (256 dual-pol antennas,
    64 channels, 64 x 64, 200 samples, 20 sources, loss |I - M|^2 with M the
    model image of the same sources): the analytic gradient against central
    differences on 16 seeded (c, p, a) -- each evaluated on its own channel's
    loss, the only one g[c] enters -- and against 4 directional derivatives of
    the whole loss (two along directions shared by all channels, as when the
    gains are shared over channels, two along directions over every (c, p, a))."""
    inp = synth.config5()
    src = inp.sources
    N, C = inp.grid_n, inp.n_chan
    model = oracle.model_image(inp.xy_m, inp.freq_hz, N, inp.n_time, src["lm"],
                               src["amp"] ** 2, src["noise_sigma"])
    g = inp.gains.astype(np.complex128)
    img = oracle.image_from(inp)
    gam = oracle.l2_loss_grad_image(img, model)
    grad = oracle.grad_gains(inp.xy_m, inp.freq_hz, g, inp.efield, N, gam)
    rng = _rng(505)
    coords = [(int(rng.integers(C)), int(rng.integers(2)), int(rng.integers(256)))
              for _ in range(16)]
    fd = []
    for c, p, a in coords:
        def loss_c(gc, c=c):
            im = oracle.image(inp.xy_m, inp.freq_hz[c:c + 1], gc[None], inp.efield[:, c:c + 1], N)
            return oracle.l2_loss(im, model[c:c + 1])
        fd.append(oracle.fd_grad(loss_c, g[c], [(p, a)])[0])
    an = np.array([grad[c] for c in coords])
    fd = np.array(fd)
    assert np.linalg.norm(an - fd) / np.linalg.norm(fd) < 1e-6

    def loss(gg):
        return oracle.l2_loss(oracle.image(inp.xy_m, inp.freq_hz, gg, inp.efield, N), model)
    dirs = []
    for _ in range(2):
        d = rng.normal(size=(2, 256)) + 1j * rng.normal(size=(2, 256))
        dirs.append(np.broadcast_to(d[None], g.shape).copy())
    for _ in range(2):
        dirs.append(rng.normal(size=g.shape) + 1j * rng.normal(size=g.shape))
    for d in dirs:
        num = oracle.fd_directional(loss, g, d)
        ana = float(np.sum(np.conj(d) * grad).real)
        assert abs(num - ana) <= 1e-6 * abs(ana), (num, ana)
