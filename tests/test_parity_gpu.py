"""Parity of the HIP imaging path with the FP64 oracle, element by element.

Tolerance (the bar for the float32 path): relative L2 error per
(channel, product) <= 1e-5, with XY / YX scaled by sqrt(|XX| |YY|)
(oracle.rel_errors).  The float32 transform of an int4 aperture carries an
error of order eps32 * log2(n_g) ~ 1e-6; the time sums are float64.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


def _imager(inp, staged=False, timing=False):
    from paper_1904_11422_amd import Imager
    im = Imager(inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                inp.kernel_sigma_cells, inp.cell_wavelengths, staged=staged, timing=timing)
    im.set_antennas(inp.xy_m, inp.freq_hz, kernels=inp.kernels)
    return im


def _dev(inp):
    import torch
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    return ef, g


def _run(inp, staged=False):
    import torch
    print(f"case {inp.name}: N={inp.grid_n} C={inp.n_chan} P={inp.n_pol} A={inp.n_ant} "
          f"T={inp.n_time} staged={staged}", flush=True)
    im = _imager(inp, staged)
    ef, g = _dev(inp)
    out = im.accumulate(ef, g)
    torch.cuda.synchronize()
    return out.cpu().numpy(), im


CASES = {
    "cfg1": lambda: synth.config1(),
    "n32_p2_ragged": lambda: synth.random_problem(101, 32, 64, 3, 2, 37),
    "n64_p2": lambda: synth.random_problem(102, 64, 256, 5, 2, 23),
    "n64_p1": lambda: synth.random_problem(103, 64, 100, 2, 1, 10),
    "n64_p2_A300": lambda: synth.random_problem(104, 64, 300, 2, 2, 6, fill=0.48),
    "n32_p2_A150": lambda: synth.random_problem(105, 32, 150, 2, 2, 5, fill=0.45),
    "cfg2_small": lambda: synth.config2(n_time=40, n_chan=4),
    "single_antenna": lambda: synth.random_problem(106, 64, 1, 2, 2, 9),
    "one_sample": lambda: synth.random_problem(107, 64, 256, 3, 2, 1),
    "n128_p2_ragged": lambda: synth.random_problem(109, 128, 400, 2, 2, 7, fill=0.45),
    "n128_p2_A1024": lambda: synth.random_problem(110, 128, 1024, 2, 2, 3, fill=0.47),
    # one polarisation at 128^2: one, two (A = 1024) and four (A = 2000) bytes per thread
    "n128_p1_ragged": lambda: synth.random_problem(119, 128, 300, 3, 1, 7, fill=0.45),
    "n128_p1_A1024": lambda: synth.random_problem(120, 128, 1024, 2, 1, 5, fill=0.47),
    "n128_p1_A2000": lambda: synth.random_problem(121, 128, 2000, 1, 1, 3, fill=0.48),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("staged", [False, True])
def test_image_matches_oracle(name, staged):
    inp = CASES[name]()
    got, _ = _run(inp, staged)
    ref = oracle.image_from(inp)
    err = oracle.rel_errors(got, ref)
    assert np.all(np.isfinite(got))
    assert err.max() <= TOL_FP32, f"max rel err {err.max():.3e}"
    if inp.n_pol == 2:
        assert np.array_equal(got[:, 2], np.conj(got[:, 1]))
        assert np.all(got[:, 0].imag == 0) and np.all(got[:, 3].imag == 0)


def test_grid128_routes():
    """128^2: one and two polarisations run the fused kernel; the staged flag
    takes the staged kernels."""
    inp = synth.random_problem(108, 128, 400, 2, 2, 3, fill=0.45)
    got, im = _run(inp, staged=False)
    assert im.last_kernel_name() == "fused_image128_kernel"
    assert oracle.rel_errors(got, oracle.image_from(inp)).max() <= TOL_FP32
    inp1 = synth.random_problem(112, 128, 300, 2, 1, 3, fill=0.45)
    got1, im1 = _run(inp1, staged=False)
    assert im1.last_kernel_name() == "fused_image128_kernel"
    assert oracle.rel_errors(got1, oracle.image_from(inp1)).max() <= TOL_FP32
    got2, im2 = _run(inp1, staged=True)
    assert im2.last_kernel_name() == "staged_fft_kernel"
    assert oracle.rel_errors(got2, oracle.image_from(inp1)).max() <= TOL_FP32


WIDE = {
    # apertures wider than N/2 cells at N = 64 (up to 48): the wide fused kernel
    "p2_a200": lambda: synth.random_problem(131, 64, 200, 3, 2, 9, fill=0.7),
    "p1_a150_ragged": lambda: synth.random_problem(132, 64, 150, 2, 1, 13, fill=0.6),
    "p2_a600_four_per_thread": lambda: synth.random_problem(133, 64, 600, 2, 2, 4, fill=0.62),
    "deployment_ellipse_55mhz": lambda: synth.deployment(134, n_time=30),
}


@pytest.mark.parametrize("name", list(WIDE))
def test_wide_aperture_matches_oracle_and_staged(name):
    """Apertures of 33-48 cells at N = 64 run the wide fused kernel (two row
    passes, inputs of rows and columns < 48); the image matches the oracle and
    the staged kernels, which handled such apertures before."""
    inp = WIDE[name]()
    got, im = _run(inp, staged=False)
    assert im.last_kernel_name() == "fused_wide_image_kernel"
    err = oracle.rel_errors(got, oracle.image_from(inp))
    print(f"  max rel err {err.max():.3e}", flush=True)
    assert err.max() <= TOL_FP32, f"{err.max():.3e}"
    got2, im2 = _run(inp, staged=True)
    assert im2.last_kernel_name() == "staged_fft_kernel"
    assert oracle.rel_errors(got, got2).max() <= TOL_FP32
    if inp.n_pol == 2:
        assert np.array_equal(got[:, 2], np.conj(got[:, 1]))


def test_timing_history_reads_every_call():
    """epic_timing_history: the main-kernel times of a run of calls, read after
    the run without a wait per call, imaging and gradient calls alike; the
    last one is the kernel that epic_last_timing reports."""
    import torch
    from paper_1904_11422_amd import _lib
    inp = synth.random_problem(140, 64, 200, 3, 2, 20)
    im = _imager(inp, timing=True)
    ef, g = _dev(inp)
    with pytest.raises(_lib.EpicError):
        im.timing_history(1)                    # no timed call yet
    img = im.accumulate(ef, g)
    gam = torch.ones_like(img)
    for _ in range(3):
        im.accumulate(ef, g, image=img)
        im.backward(ef, g, gam)
    hist = im.timing_history(7)
    print(f"  history {hist}", flush=True)
    assert len(hist) == 7 and all(h > 0 for h in hist)
    last = im.last_timing()[0]
    assert abs(hist[-1] - last) <= 0.05 * last + 0.01
    with pytest.raises(_lib.EpicError):
        im.timing_history(8)                    # seven timed calls so far
    with pytest.raises(_lib.EpicError):
        im.timing_history(257)
    im.close()


def test_wide_aperture_is_deterministic_and_continues():
    import torch
    inp = synth.random_problem(135, 64, 180, 2, 2, 10, fill=0.66)
    im = _imager(inp)
    ef, g = _dev(inp)
    a = im.accumulate(ef, g).cpu().numpy()
    b = im.accumulate(ef, g).cpu().numpy()
    assert im.last_kernel_name() == "fused_wide_image_kernel"
    assert np.array_equal(a, b)
    out = im.accumulate(ef[:3], g)
    im.accumulate(ef[3:], g, image=out, reset=False)
    torch.cuda.synchronize()
    assert oracle.rel_errors(out.cpu().numpy(), oracle.image_from(inp)).max() <= TOL_FP32


def test_reset_zero_continues_integration():
    import torch
    inp = synth.random_problem(111, 64, 128, 3, 2, 17)
    im = _imager(inp)
    ef, g = _dev(inp)
    img = im.accumulate(ef[:6], g)
    im.accumulate(ef[6:], g, image=img, reset=False)
    torch.cuda.synchronize()
    ref = oracle.image_from(inp)
    assert oracle.rel_errors(img.cpu().numpy(), ref).max() <= TOL_FP32


def test_reset_zero_continues_integration_n128():
    """128^2: reset=0 adds to the image, and the two column halves of a
    sample land in their own pixels (split across calls and segments)."""
    import torch
    inp = synth.random_problem(117, 128, 512, 2, 2, 9, fill=0.45)
    im = _imager(inp)
    ef, g = _dev(inp)
    img = im.accumulate(ef[:4], g)
    im.accumulate(ef[4:], g, image=img, reset=False)
    torch.cuda.synchronize()
    assert im.last_kernel_name() == "fused_image128_kernel"
    assert oracle.rel_errors(img.cpu().numpy(), oracle.image_from(inp)).max() <= TOL_FP32


def test_reset_zero_continues_integration_n128_one_pol():
    import torch
    inp = synth.random_problem(122, 128, 600, 3, 1, 10, fill=0.45)
    im = _imager(inp)
    ef, g = _dev(inp)
    img = im.accumulate(ef[:3], g)
    im.accumulate(ef[3:], g, image=img, reset=False)
    torch.cuda.synchronize()
    assert im.last_kernel_name() == "fused_image128_kernel"
    assert oracle.rel_errors(img.cpu().numpy(), oracle.image_from(inp)).max() <= TOL_FP32


@pytest.mark.parametrize("P", [1, 2])
def test_bitwise_deterministic_n128(P):
    import torch
    inp = synth.random_problem(118, 128, 700, 2, P, 11, fill=0.45)
    im = _imager(inp)
    ef, g = _dev(inp)
    a = im.accumulate(ef, g).clone()
    b = im.accumulate(ef, g)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_bitwise_deterministic():
    import torch
    inp = synth.random_problem(112, 64, 256, 4, 2, 31)
    im = _imager(inp)
    ef, g = _dev(inp)
    a = im.accumulate(ef, g).clone()
    b = im.accumulate(ef, g)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_fewer_samples_than_workgroups():
    """C*T below the persistent grid: every workgroup still owns >= 1 sample."""
    inp = synth.random_problem(113, 64, 64, 2, 2, 3)
    got, _ = _run(inp)
    assert oracle.rel_errors(got, oracle.image_from(inp)).max() <= TOL_FP32


@pytest.mark.parametrize("seed,C,T", [
    (821, 5, 1),      # one unit per workgroup: nothing staged ahead
    (822, 3, 2),      # two units: staged ahead, nothing prefetched
    (823, 600, 1),    # more channels than workgroups: the next unit's gains reloaded
    (824, 300, 3),    # parts crossing channels inside a workgroup's range
    (825, 2, 257),    # ragged parts of 64-65 samples (teams of 4)
    (826, 1, 1100),   # parts of 137-138 samples (teams of 8): float64 flushes
])
def test_one_barrier_form_edges(seed, C, T):
    """The double-buffered one-barrier form (N = 64, two polarisations, at most
    256 antennas, Gaussian taps) at its edges: workgroups with one or two
    units, units whose successor is in another channel, and parts longer than
    the float32 block.  The image matches the oracle, and a second call with
    reset = 0 adds the same samples again."""
    import torch
    inp = synth.random_problem(seed, 64, 200, C, 2, T, fill=0.45)
    im = _imager(inp)
    ef, g = _dev(inp)
    got = im.accumulate(ef, g)
    torch.cuda.synchronize()
    assert im.last_kernel_name() == "fused_image_kernel"
    ref = oracle.image_from(inp)
    err = oracle.rel_errors(got.cpu().numpy(), ref)
    print(f"  max rel err {err.max():.3e}", flush=True)
    assert err.max() <= TOL_FP32, f"{err.max():.3e}"
    im.accumulate(ef, g, image=got, reset=False)
    torch.cuda.synchronize()
    assert oracle.rel_errors(got.cpu().numpy(), 2.0 * ref).max() <= TOL_FP32


def test_fused_and_staged_agree():
    inp = synth.random_problem(114, 64, 256, 3, 2, 20)
    a, _ = _run(inp, staged=False)
    b, _ = _run(inp, staged=True)
    assert oracle.rel_errors(a, b).max() <= 2 * TOL_FP32


def test_offgrid_geometry_is_rejected_and_previous_kept():
    from paper_1904_11422_amd import EpicError
    inp = synth.random_problem(115, 32, 16, 1, 1, 4)
    im = _imager(inp)
    far = inp.xy_m.copy()
    far[0, 0] = 1e4
    with pytest.raises(EpicError, match="OFFGRID"):
        im.set_antennas(far, inp.freq_hz)
    ef, g = _dev(inp)
    got = im.accumulate(ef, g).cpu().numpy()
    assert oracle.rel_errors(got, oracle.image_from(inp)).max() <= TOL_FP32


def test_invalid_calls_leave_output_untouched():
    import torch
    from paper_1904_11422_amd import EpicError, Imager
    inp = synth.random_problem(116, 32, 16, 1, 1, 4)
    im = Imager(32, 1, 1, 16)
    ef, g = _dev(inp)
    with pytest.raises(EpicError, match="STATE"):
        im.accumulate(ef, g)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    out = torch.full((1, 1, 32, 32), 7.0, dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        im.accumulate(ef[:, :, :, :8], g, image=out)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)


def test_empty_integration_is_rejected_and_output_untouched():
    import torch
    from paper_1904_11422_amd import EpicError
    inp = synth.random_problem(119, 64, 64, 2, 2, 3)
    im = _imager(inp)
    ef, g = _dev(inp)
    out = torch.full(im.image_shape(), 3.0, dtype=torch.complex128, device="cuda")
    with pytest.raises(EpicError, match="INVALID"):
        im.accumulate(ef[:0], g, image=out)
    torch.cuda.synchronize()
    assert torch.all(out == 3.0)


@pytest.mark.slow
def test_config2_full_size_sampled_channels():
    """The benchmark's launch (C=132, T=1000) checked on sampled channels, each
    against the oracle over all 1000 samples."""
    import torch
    inp = synth.config2()
    got, _ = _run(inp)
    for c in (0, 65, 131):
        sub = synth.Inputs(inp.grid_n, 1, inp.n_pol, inp.n_ant, 3, 0.5, 0.5, inp.xy_m,
                           inp.freq_hz[c:c + 1], inp.gains[c:c + 1], inp.efield[:, c:c + 1])
        ref = oracle.image_from(sub)
        err = oracle.rel_errors(got[c:c + 1], ref)
        assert err.max() <= TOL_FP32, f"channel {c}: {err.max():.3e}"
    # properties that hold for every channel
    assert np.all(got[:, 0].real >= 0) and np.all(got[:, 3].real >= 0)
    assert np.all(np.abs(got[:, 1]) ** 2 <= got[:, 0].real * got[:, 3].real * (1 + 1e-5) + 1e-3)
    del torch


@pytest.mark.parametrize("seed,N,A,C,P,T,fill,route", [
    (801, 128, 4096, 1, 2, 2, 0.9, "staged_fft_kernel"),     # the largest antenna count taken
    (802, 64, 1024, 2, 1, 3, 0.48, "fused_image_kernel"),    # 2 samples per thread
    (804, 64, 1024, 2, 2, 3, 0.48, "fused_image_kernel"),    # 4 samples per thread, all used
    (803, 64, 2048, 1, 2, 2, 0.9, "staged_fft_kernel"),      # beyond 4 samples per thread
])
def test_maximum_antenna_counts(seed, N, A, C, P, T, fill, route):
    """The largest configurations: A = 4096 (the limit), and the switch from
    the fused kernels to the staged ones once a thread would hold more than
    four samples or the aperture leaves N/2 cells."""
    inp = synth.random_problem(seed, N, A, C, P, T, fill=fill)
    got, im = _run(inp)
    assert im.last_kernel_name() == route
    assert oracle.rel_errors(got, oracle.image_from(inp)).max() <= TOL_FP32


@pytest.mark.parametrize("seed,A,C,T,K,cpx", [
    (811, 513, 2, 7, 3, False),     # one past two bytes per thread
    (812, 1000, 2, 131, 3, False),  # float64 flushes after 128 samples, ragged
    (813, 900, 2, 5, 7, True),      # complex 7 x 7 kernels: step lists read in chunks
])
def test_many_antennas_stage_in_the_grid_rows(seed, A, C, T, K, cpx):
    """More than 512 dual-pol antennas at N = 64 (four sample bytes per
    thread): E' is staged in the second polarisation's grid rows N/2 .. N-1,
    whose column transforms exchange through the first polarisation's
    columns instead, so that two workgroups share a CU.  The image matches
    the oracle, and the Hermitian pair XY = conj(YX) holds exactly."""
    inp = synth.random_problem(seed, 64, A, C, 2, T, fill=0.42 if K > 3 else 0.48)
    if cpx:
        inp = synth.with_kernels(inp, K, seed + 7)
    got, im = _run(inp)
    assert im.last_kernel_name() == "fused_image_kernel"
    err = oracle.rel_errors(got, oracle.image_from(inp))
    print(f"  max rel err {err.max():.3e}", flush=True)
    assert err.max() <= TOL_FP32, f"{err.max():.3e}"
    assert np.array_equal(got[:, 2], np.conj(got[:, 1]))


def test_antenna_limit_is_enforced():
    from paper_1904_11422_amd import EpicError, Imager
    with pytest.raises(EpicError, match="INVALID"):
        Imager(64, 1, 2, 4097)
