"""The no-allocation imaging call (epic_image_accumulate_noalloc) against the
ordinary one (epic_image_accumulate), both through the C ABI on the same
context: two calls in a row, the second with fewer samples, at the float32
bar of the parity tests (relative L2 per (channel, product) <= 1e-5).  Both
calls run the same kernels with the same persistent grid and reduction
order, so the images are also compared bit for bit."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


def _setup(inp, **kw):
    import torch
    from paper_1904_11422_amd import Imager
    im = Imager(inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                inp.kernel_sigma_cells, inp.cell_wavelengths, **kw)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    return im, ef, g


def _call(im, name, ef, n_time, g, img, reset=1):
    fn = getattr(im.L, name)
    return fn(im._ctx, ctypes.c_void_p(ef.data_ptr()), int(n_time), ctypes.c_void_p(g.data_ptr()),
              ctypes.c_void_p(img.data_ptr()), reset)


CASES = {
    # the LWA-like shape with fewer channels and samples (two sample bytes per
    # 512-thread workgroup pass), a ragged N = 32 case, N = 128 at one and
    # two polarisations, and wide apertures at N = 64 (the deployed ellipse
    # runs transposed in a 40-row block)
    "n64_p2_lwa": lambda: synth.config2(n_time=120, n_chan=12),
    "n32_p2_ragged": lambda: synth.random_problem(901, 32, 64, 3, 2, 37),
    "n128_p2": lambda: synth.random_problem(902, 128, 400, 2, 2, 9, fill=0.45),
    "n128_p1": lambda: synth.random_problem(903, 128, 300, 3, 1, 7, fill=0.45),
    "n64_wide": lambda: synth.random_problem(904, 64, 200, 2, 2, 11, fill=0.62),
    "n64_wide_transposed": lambda: synth.deployment(906, n_time=14, n_chan=3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_noalloc_matches_accumulate_twice(case):
    import torch
    from paper_1904_11422_amd import _lib
    inp = CASES[case]()
    print(f"case {case}: N={inp.grid_n} C={inp.n_chan} P={inp.n_pol} A={inp.n_ant} T={inp.n_time}",
          flush=True)
    im, ef, g = _setup(inp)
    T = inp.n_time
    for n_time in (T, max(1, T // 3)):             # the second call is smaller
        ref = torch.empty(im.image_shape(), dtype=torch.complex128, device="cuda")
        got = torch.full(im.image_shape(), float("nan"), dtype=torch.complex128, device="cuda")
        _lib.check(im.L, im._ctx, _call(im, "epic_image_accumulate", ef, n_time, g, ref))
        _lib.check(im.L, im._ctx, _call(im, "epic_image_accumulate_noalloc", ef, n_time, g, got))
        torch.cuda.synchronize()
        a, b = got.cpu().numpy(), ref.cpu().numpy()
        err = oracle.rel_errors(a, b).max()
        print(f"  n_time={n_time}: rel err vs epic_image_accumulate {err:.3e}", flush=True)
        assert err <= TOL_FP32, f"{err:.3e}"
        assert np.array_equal(a, b)
    # the second call against the oracle on its first channel
    n_time = max(1, T // 3)
    want = oracle.image(inp.xy_m, inp.freq_hz[:1], inp.gains[:1], inp.efield[:n_time, :1], inp.grid_n)
    assert oracle.rel_errors(a[:1], want).max() <= TOL_FP32
    im.close()


def test_noalloc_continues_an_integration():
    """reset = 0 adds to the caller's image, as epic_image_accumulate does."""
    import torch
    from paper_1904_11422_amd import _lib
    inp = synth.random_problem(905, 64, 150, 3, 2, 30)
    im, ef, g = _setup(inp)
    ref = torch.empty(im.image_shape(), dtype=torch.complex128, device="cuda")
    got = torch.empty_like(ref)
    _lib.check(im.L, im._ctx, _call(im, "epic_image_accumulate", ef, 30, g, ref))
    _lib.check(im.L, im._ctx, _call(im, "epic_image_accumulate_noalloc", ef[:18], 18, g, got))
    _lib.check(im.L, im._ctx, _call(im, "epic_image_accumulate_noalloc", ef[18:], 12, g, got, reset=0))
    torch.cuda.synchronize()
    assert oracle.rel_errors(got.cpu().numpy(), ref.cpu().numpy()).max() <= TOL_FP32
    im.close()


def test_noalloc_refusals_leave_the_image_untouched():
    """The staged path, and a call whose slots exceed the static array, are
    refused before anything is enqueued."""
    import torch
    from paper_1904_11422_amd import _lib
    inp = synth.random_problem(906, 64, 100, 2, 2, 4)
    im, ef, g = _setup(inp, staged=True)
    img = torch.full(im.image_shape(), 3.0 + 1j, dtype=torch.complex128, device="cuda")
    st = _call(im, "epic_image_accumulate_noalloc", ef, 4, g, img)
    assert st == _lib.EPIC_E_UNSUPPORTED
    assert b"fused" in im.L.epic_last_error(im._ctx)
    im.close()
    # N = 128, P = 2, 200 channels: (W + 2C - 1) slots of 256 KiB, far past 96 MiB
    inp = synth.random_problem(907, 128, 64, 200, 2, 2, fill=0.3)
    im, ef, g = _setup(inp)
    img = torch.full(im.image_shape(), 3.0 + 1j, dtype=torch.complex128, device="cuda")
    st = _call(im, "epic_image_accumulate_noalloc", ef, 2, g, img)
    assert st == _lib.EPIC_E_UNSUPPORTED
    assert b"static scratch" in im.L.epic_last_error(im._ctx)
    torch.cuda.synchronize()
    assert bool((img == (3.0 + 1j)).all())
    im.close()
