"""User complex gridding kernels per channel and antenna (epic_set_antennas_kernels),
supports up to 15 x 15, against the FP64 oracle gridding with the same
kernels.  Bars as for the Gaussian: 1e-5 relative per (channel, product) for
the float32 paths, 1e-3 for the split forms, 1e-4 for gradients."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_GRAD = 1e-4


def _imager(inp, **kw):
    from paper_1904_11422_amd import Imager
    im = Imager(inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                inp.kernel_sigma_cells, inp.cell_wavelengths, **kw)
    im.set_antennas(inp.xy_m, inp.freq_hz, kernels=inp.kernels)
    return im


def _dev(inp):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda(),
            torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda())


def _case(seed, N, A, C, P, T, K, fill):
    return synth.with_kernels(synth.random_problem(seed, N, A, C, P, T, fill=fill), K, seed + 1)


CASES = {
    # name: (inputs, imager options, expected main kernel)
    "n32_p2_k3": (lambda: _case(601, 32, 48, 2, 2, 9, 3, 0.45), {}, "fused_image_kernel"),
    "n64_p2_k7": (lambda: _case(602, 64, 96, 2, 2, 7, 7, 0.38), {}, "fused_image_kernel"),
    "n64_p1_k5": (lambda: _case(603, 64, 120, 3, 1, 6, 5, 0.4), {}, "fused_image_kernel"),
    "n128_p2_k9": (lambda: _case(604, 128, 300, 2, 2, 4, 9, 0.38), {}, "fused_image128_kernel"),
    "n128_p2_k15": (lambda: _case(605, 128, 200, 1, 2, 3, 15, 0.25), {}, "fused_image128_kernel"),
    "n128_p1_k7": (lambda: _case(609, 128, 400, 2, 1, 4, 7, 0.4), {}, "fused_image128_kernel"),
    "n64_p2_k11_wide": (lambda: _case(606, 64, 80, 2, 2, 5, 11, 0.45), {}, "fused_wide_image_kernel"),
    "n64_p1_k15_beyond_wide": (lambda: _case(610, 64, 60, 2, 1, 4, 15, 0.6), {}, "staged_fft_kernel"),
    "n32_p2_k5_staged": (lambda: _case(607, 32, 40, 2, 2, 6, 5, 0.4), {"staged": True},
                         "staged_fft_kernel"),
    "split16_p2_k5": (lambda: _case(608, 32, 16, 2, 2, 40, 5, 0.4), {"precision": "split_fp16"},
                      "split_image_kernel"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_complex_kernels_match_oracle(name):
    import torch
    make, kw, kname = CASES[name]
    inp = make()
    print(f"case {name}: N={inp.grid_n} C={inp.n_chan} P={inp.n_pol} A={inp.n_ant} "
          f"K={inp.kernel_support} T={inp.n_time} {kw}", flush=True)
    im = _imager(inp, **kw)
    ef, g = _dev(inp)
    got = im.accumulate(ef, g).cpu().numpy()
    torch.cuda.synchronize()
    assert im.last_kernel_name() == kname
    err = oracle.rel_errors(got, oracle.image_from(inp))
    print(f"  max rel err {err.max():.3e}")
    assert err.max() <= (1e-3 if "split" in name else TOL_FP32), f"{err.max():.3e}"
    if inp.n_pol == 2:
        assert np.array_equal(got[:, 2], np.conj(got[:, 1]))


def test_complex_kernels_are_deterministic_and_continue():
    """Bitwise-identical repeats; reset = 0 continues the integration."""
    import torch
    inp = _case(611, 64, 64, 2, 2, 12, 5, 0.4)
    im = _imager(inp)
    ef, g = _dev(inp)
    a = im.accumulate(ef, g).cpu().numpy()
    b = im.accumulate(ef, g).cpu().numpy()
    assert np.array_equal(a, b)
    out = im.accumulate(ef[:5], g)
    im.accumulate(ef[5:], g, image=out, reset=False)
    torch.cuda.synchronize()
    assert oracle.rel_errors(out.cpu().numpy(), oracle.image_from(inp)).max() <= TOL_FP32


def test_gaussian_given_as_kernels_matches_the_built_in_path():
    """The built-in Gaussian, passed back in as (real) kernels, gives the image
    of epic_set_antennas (the complex-kernel kernels may partition the samples
    differently, so agreement is to float32 summation order, not bitwise)."""
    import torch
    inp = synth.random_problem(612, 64, 100, 2, 2, 6)
    X, Y = oracle.antenna_cells(inp.xy_m, inp.freq_hz, 64)
    _, _, w = oracle.kernel_taps(X, Y, 64, 3, 0.5)
    kern = w.reshape(2, 100, 3, 3).astype(np.complex64)
    from paper_1904_11422_amd import Imager
    a_im = Imager(64, 2, 2, 100)
    a_im.set_antennas(inp.xy_m, inp.freq_hz)
    b_im = Imager(64, 2, 2, 100)
    b_im.set_antennas(inp.xy_m, inp.freq_hz, kernels=kern)
    ef, g = _dev(inp)
    a = a_im.accumulate(ef, g).cpu().numpy()
    b = b_im.accumulate(ef, g).cpu().numpy()
    torch.cuda.synchronize()
    assert oracle.rel_errors(b, a).max() <= 1e-6


@pytest.mark.parametrize("seed,N,A,C,P,T,K", [(621, 32, 16, 2, 2, 5, 5), (622, 32, 20, 1, 1, 7, 3),
                                              (627, 64, 90, 2, 2, 4, 9),
                                              (623, 64, 96, 2, 2, 6, 7), (624, 64, 50, 2, 1, 4, 9),
                                              (625, 128, 150, 1, 2, 3, 7), (626, 128, 120, 2, 1, 3, 11)])
def test_complex_kernel_gradient_matches_oracle(seed, N, A, C, P, T, K):
    import torch
    inp = _case(seed, N, A, C, P, T, K, 0.35)
    print(f"case N={N} A={A} C={C} P={P} T={T} K={K}", flush=True)
    im = _imager(inp)
    ef, g = _dev(inp)
    img = im.accumulate(ef, g).cpu().numpy()
    rng = np.random.default_rng(seed)
    gam = oracle.l2_loss_grad_image(img, img * (1 + 0.05 * rng.normal(size=img.shape)))
    got = im.backward(ef, g, torch.from_numpy(gam).cuda()).cpu().numpy()
    ref = oracle.grad_gains(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, N, gam, K,
                            kernels=inp.kernels)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= TOL_GRAD, f"{rel:.3e}"


def test_complex_kernels_refusals():
    from paper_1904_11422_amd import EpicError, Imager
    inp = _case(631, 32, 16, 1, 2, 3, 3, 0.4)
    with pytest.raises(EpicError, match="UNSUPPORTED"):
        Imager(32, 1, 2, 16, kernel_support=9, remove_autos=True)
    bad = inp.kernels.copy()
    bad[0, 0, 1, 1] = np.nan
    with pytest.raises(EpicError, match="INVALID"):
        Imager(32, 1, 2, 16).set_antennas(inp.xy_m, inp.freq_hz, kernels=bad)
