"""Gain gradient of the HIP adjoint kernel against the FP64 oracle's analytic
gradient (itself pinned to finite differences) and against central finite
differences of the GPU forward image.

Bar: relative L2 error of the gradient <= 1e-4.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-4


def _setup(inp):
    import torch
    from paper_1904_11422_amd import Imager
    print(f"case {inp.name}: N={inp.grid_n} C={inp.n_chan} P={inp.n_pol} A={inp.n_ant} "
          f"T={inp.n_time}", flush=True)
    im = Imager(inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                inp.kernel_sigma_cells, inp.cell_wavelengths)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    return im, ef, g


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("seed,N,A,C,P,T", [(201, 32, 16, 2, 2, 5), (202, 32, 16, 1, 1, 7),
                                          (203, 64, 256, 3, 2, 11), (204, 64, 90, 2, 1, 4),
                                          # 128^2: one, two and four sample bytes per thread
                                          (206, 128, 200, 2, 2, 3), (207, 128, 300, 3, 1, 4),
                                          (208, 128, 1024, 1, 2, 2), (209, 128, 1024, 2, 1, 3)])
def test_grad_matches_oracle_l2_loss(seed, N, A, C, P, T):
    import torch
    inp = synth.random_problem(seed, N, A, C, P, T, fill=0.45)
    im, ef, g = _setup(inp)
    img = im.accumulate(ef, g).cpu().numpy()
    rng = np.random.default_rng(seed)
    model = img * (1 + 0.05 * rng.normal(size=img.shape))         # any fixed M
    gam = oracle.l2_loss_grad_image(img, model)
    got = im.backward(ef, g, torch.from_numpy(gam).cuda()).cpu().numpy()
    ref = oracle.grad_gains(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, N, gam)
    assert _rel(got, ref) <= TOL_GRAD, f"{_rel(got, ref):.3e}"


@pytest.mark.parametrize("seed,N,A,C,P,T,fill,staged", [
    (232, 32, 40, 2, 1, 9, 0.7, False),
    (233, 64, 256, 2, 2, 5, 0.45, True),     # EPIC_FLAG_STAGED
    (234, 128, 300, 1, 1, 3, 0.45, True),
])
def test_staged_grad_matches_oracle(seed, N, A, C, P, T, fill, staged):
    """The gradient on the staged kernels (batches of the forward stages, then
    the adjoint stages) against the oracle."""
    import torch
    from paper_1904_11422_amd import Imager
    inp = synth.random_problem(seed, N, A, C, P, T, fill=fill)
    print(f"case {seed}: N={N} A={A} C={C} P={P} T={T} fill={fill} staged={staged}", flush=True)
    im = Imager(N, C, P, A, staged=staged)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    img = im.accumulate(ef, g)
    assert im.last_kernel_name() == "staged_fft_kernel"
    img = img.cpu().numpy()
    rng = np.random.default_rng(seed)
    gam = oracle.l2_loss_grad_image(img, img * (1 + 0.05 * rng.normal(size=img.shape)))
    got = im.backward(ef, g, torch.from_numpy(gam).cuda()).cpu().numpy()
    assert im.last_kernel_name() == "staged_degrid_kernel"
    ref = oracle.grad_gains(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, N, gam)
    assert _rel(got, ref) <= TOL_GRAD, f"{_rel(got, ref):.3e}"


def test_staged_grad_spans_batches():
    """More samples than one staged batch: the float64 sums carry across batches."""
    import torch
    from paper_1904_11422_amd import Imager
    inp = synth.random_problem(235, 32, 24, 2, 2, 150, fill=0.7)
    im = Imager(32, 2, 2, 24)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    img = im.accumulate(ef, g).cpu().numpy()
    rng = np.random.default_rng(235)
    gam = oracle.l2_loss_grad_image(img, img * (1 + 0.05 * rng.normal(size=img.shape)))
    got = im.backward(ef, g, torch.from_numpy(gam).cuda()).cpu().numpy()
    ref = oracle.grad_gains(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 32, gam)
    assert _rel(got, ref) <= TOL_GRAD, f"{_rel(got, ref):.3e}"


def test_grad_cross_products_only():
    """Upstream gradient on XY and YX alone exercises the h terms."""
    import torch
    inp = synth.random_problem(205, 32, 24, 2, 2, 6)
    im, ef, g = _setup(inp)
    rng = np.random.default_rng(3)
    gam = np.zeros((2, 4, 32, 32), complex)
    gam[:, 1] = rng.normal(size=(2, 32, 32)) + 1j * rng.normal(size=(2, 32, 32))
    gam[:, 2] = rng.normal(size=(2, 32, 32)) + 1j * rng.normal(size=(2, 32, 32))
    got = im.backward(ef, g, torch.from_numpy(gam).cuda()).cpu().numpy()
    ref = oracle.grad_gains(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 32, gam)
    assert _rel(got, ref) <= TOL_GRAD


def test_grad_matches_finite_differences_of_gpu_forward():
    """Central differences of the GPU image (float64 loss of float64 sums)."""
    import torch
    inp = synth.random_problem(206, 32, 8, 1, 2, 4)
    im, ef, g = _setup(inp)
    rng = np.random.default_rng(4)
    w = rng.normal(size=(1, 4, 32, 32))

    def loss(gg):
        out = im.accumulate(ef, torch.from_numpy(gg.astype(np.complex64)).cuda()).cpu().numpy()
        return float(np.sum(w * out.real))
    gam = w.astype(complex)                                         # dL/dRe(I)
    got = im.backward(ef, g, torch.from_numpy(gam).cuda()).cpu().numpy()
    g0 = inp.gains.astype(np.complex128)
    coords = [(0, 0, 1), (0, 1, 5), (0, 0, 7), (0, 1, 0)]
    fd = oracle.fd_grad(loss, g0, coords, rel_step=2e-3)
    an = np.array([got[c] for c in coords])
    assert _rel(an, fd) <= 5e-3


def test_config5_gradient_and_autograd():
    """Calibration setup (model image from point sources, loss |I - M|^2) through
    the autograd Function with gains shared over channels."""
    import torch
    from paper_1904_11422_amd import image
    inp = synth.config5(n_time=40, n_chan=4, n_src=8)
    im, ef, _ = _setup(inp)
    src = inp.sources
    model = oracle.model_image(inp.xy_m, inp.freq_hz, 64, inp.n_time, src["lm"],
                               src["amp"] ** 2, src["noise_sigma"])
    g_pa = torch.from_numpy(src["g_eval"]).cuda().requires_grad_(True)       # [P, A]
    gains = g_pa[None].expand(inp.n_chan, 2, 256)
    img = image(im, gains, ef)
    m = torch.from_numpy(model).cuda()
    loss = ((img - m).abs() ** 2).sum()
    loss.backward()
    got = g_pa.grad.cpu().numpy()
    img_np = img.detach().cpu().numpy()
    gam = oracle.l2_loss_grad_image(img_np, model)
    ref = oracle.grad_gains(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 64, gam).sum(0)
    assert _rel(got, ref) <= TOL_GRAD, f"{_rel(got, ref):.3e}"
    ref_img = oracle.image_from(inp)
    assert oracle.rel_errors(img_np, ref_img).max() <= 1e-5


def test_config5_full_shape_gradient():
    """The calibration workload at its full shape (256 dual-pol antennas,
    64 channels, 64 x 64, 200 samples, 20 sources): gains shared over channels
    through the autograd Function, loss |I - M|^2 with M the oracle's model image
    of the same sources.  The gradient against the oracle's (pinned to finite
    differences at this shape) within 1e-4, the image against the oracle on
    sampled channels within 1e-5."""
    import torch
    from paper_1904_11422_amd import image
    inp = synth.config5()
    im, ef, _ = _setup(inp)
    src = inp.sources
    model = oracle.model_image(inp.xy_m, inp.freq_hz, 64, inp.n_time, src["lm"],
                               src["amp"] ** 2, src["noise_sigma"])
    g_pa = torch.from_numpy(src["g_eval"]).cuda().requires_grad_(True)       # [P, A]
    img = image(im, g_pa[None].expand(inp.n_chan, 2, 256), ef)
    loss = ((img - torch.from_numpy(model).cuda()).abs() ** 2).sum()
    loss.backward()
    assert im.last_kernel_name() == "adjoint_kernel"
    got = g_pa.grad.cpu().numpy()
    img_np = img.detach().cpu().numpy()
    gam = oracle.l2_loss_grad_image(img_np, model)
    ref = oracle.grad_gains(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 64, gam).sum(0)
    err = _rel(got, ref)
    print(f"config5 gradient rel err {err:.3e}", flush=True)
    assert err <= TOL_GRAD, f"{err:.3e}"
    for c in (0, 31, 63):
        ref_c = oracle.image(inp.xy_m, inp.freq_hz[c:c + 1], inp.gains[c:c + 1],
                             inp.efield[:, c:c + 1], 64)
        assert oracle.rel_errors(img_np[c:c + 1], ref_c).max() <= 1e-5


@pytest.mark.parametrize("seed,A,C,P,T,fill,K", [(231, 120, 2, 2, 7, 0.62, 3), (241, 90, 2, 1, 9, 0.7, 3),
                                                 (242, 600, 1, 2, 3, 0.62, 3), (243, 80, 2, 2, 5, 0.45, 11),
                                                 (244, 256, 2, 2, 6, None, 3)])
def test_wide_grad_matches_oracle(seed, A, C, P, T, fill, K):
    """Apertures of 33-48 cells at N = 64: the wide fused image and its adjoint
    (adjoint_wide_kernel) against the oracle's gradient; K > 3 with complex
    kernels.  The cases cover wide blocks of 40 and 48 rows, with the taps
    transposed (the narrower extent along the rows) or not; fill None is the
    deployed ellipse (40 rows, transposed)."""
    import torch
    from paper_1904_11422_amd import Imager
    if fill is None:
        inp = synth.deployment(seed, n_time=T, n_chan=C, n_pol=P)
    else:
        inp = synth.random_problem(seed, 64, A, C, P, T, fill=fill)
    if K != 3:
        inp = synth.with_kernels(inp, K, seed + 1)
    print(f"case {seed}: A={A} C={C} P={P} T={T} fill={fill} K={K}", flush=True)
    im = Imager(64, C, P, A, kernel_support=K)
    im.set_antennas(inp.xy_m, inp.freq_hz, kernels=inp.kernels)
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    img = im.accumulate(ef, g)
    assert im.last_kernel_name() == "fused_wide_image_kernel"
    img = img.cpu().numpy()
    rng = np.random.default_rng(seed)
    gam = oracle.l2_loss_grad_image(img, img * (1 + 0.05 * rng.normal(size=img.shape)))
    got = im.backward(ef, g, torch.from_numpy(gam).cuda()).cpu().numpy()
    assert im.last_kernel_name() == "adjoint_wide_kernel"
    ref = oracle.grad_gains(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 64, gam, K,
                            kernels=inp.kernels)
    assert _rel(got, ref) <= TOL_GRAD, f"{_rel(got, ref):.3e}"
