"""Post-processing on the GPU (pseudo-Stokes, kernel taper and its correction)
against the oracle.  The pseudo-Stokes arithmetic is float64 on the image:
against the oracle applied to the same GPU image, 1e-14 relative.  The taper is
float64 from the float32 kernel weights: 1e-6 of its maximum against the
oracle's float64 weights.  Chained with the imager, the float32 imaging bar
(1e-5 of each channel's I norm)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _imager(inp, **kw):
    from paper_1904_11422_amd import Imager
    im = Imager(inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                inp.kernel_sigma_cells, inp.cell_wavelengths, **kw)
    im.set_antennas(inp.xy_m, inp.freq_hz, kernels=inp.kernels)
    return im


def _run(inp, floor=None, **kw):
    import torch
    im = _imager(inp, **kw)
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    img = im.accumulate(ef, g)
    out = im.postprocess(img, floor)
    taper = im.kernel_taper()
    torch.cuda.synchronize()
    return img.cpu().numpy(), out.cpu().numpy(), taper.cpu().numpy()


CASES = {
    "n64_p2": lambda: synth.random_problem(701, 64, 128, 3, 2, 9),
    "n32_p1": lambda: synth.random_problem(702, 32, 40, 2, 1, 7),
    "n128_p2": lambda: synth.random_problem(703, 128, 300, 2, 2, 3, fill=0.45),
    "n64_p2_k5_complex": lambda: synth.with_kernels(synth.random_problem(704, 64, 60, 2, 2, 5,
                                                                          fill=0.4), 5, 705),
}


@pytest.mark.parametrize("name", list(CASES))
def test_pseudo_stokes_and_taper_match_oracle(name):
    inp = CASES[name]()
    print(f"case {name}", flush=True)
    img, st, taper = _run(inp)
    # the arithmetic on the same image
    ref_same = oracle.pseudo_stokes(img)
    assert np.max(np.abs(st - ref_same)) <= 1e-14 * np.abs(ref_same).max()
    # chained with the imager
    ref = oracle.pseudo_stokes(oracle.image_from(inp))
    nI = np.linalg.norm(ref[:, 0].reshape(inp.n_chan, -1), axis=-1)
    d = np.linalg.norm((st - ref).reshape(inp.n_chan, st.shape[1], -1), axis=-1)
    assert np.all(d <= 1e-5 * nI[:, None]), f"{np.max(d / nI[:, None]):.3e}"
    # the taper
    tref = oracle.kernel_taper(inp.xy_m, inp.freq_hz, inp.grid_n, inp.kernel_support,
                               inp.kernel_sigma_cells, inp.cell_wavelengths, inp.kernels)
    assert np.max(np.abs(taper - tref)) <= 1e-6 * tref.max()


@pytest.mark.parametrize("floor", [0.0, 1e-3, 0.05])
def test_taper_correction_matches_oracle(floor):
    inp = synth.random_problem(711, 64, 100, 2, 2, 6)
    img, st, taper = _run(inp, floor)
    tref = oracle.kernel_taper(inp.xy_m, inp.freq_hz, 64)
    want = oracle.taper_corrected(oracle.pseudo_stokes(img), taper, floor)
    assert np.max(np.abs(st - want)) <= 1e-14 * np.abs(want).max()
    # the mask agrees with the oracle's taper away from the threshold
    tm = tref.reshape(2, -1).max(axis=1)[:, None, None]
    clear = np.abs(tref - floor * tm) > 1e-5 * tm
    keep_gpu = st[:, 0] != 0
    assert np.array_equal(keep_gpu[clear], (tref >= floor * tm)[clear])


def test_taper_correction_recovers_point_kernel_image():
    """Antennas on whole cells share one Gaussian kernel: the corrected GPU image
    equals the oracle's image gridded with a unit 1 x 1 kernel.  Bar: the float32
    imaging error (~1e-6 of the image) amplified by at most 1 / floor = 100 where
    the taper is smallest."""
    N, A, T = 64, 24, 8
    inp = synth.random_problem(721, N, A, 1, 2, T)
    cell_m = oracle.C0 / inp.freq_hz[0] * 0.5
    cells = np.random.default_rng(722).choice(np.arange(-10, 11), size=(A, 2))
    inp = synth.Inputs(N, 1, 2, A, 3, 0.5, 0.5, cells * cell_m, inp.freq_hz, inp.gains,
                       inp.efield, name="whole_cells")
    floor = 1e-2
    _, st, taper = _run(inp, floor)
    point = oracle.image(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, N, 1, 0.5,
                         kernels=np.ones((1, A, 1, 1), complex))
    want = oracle.pseudo_stokes(point)
    keep = taper[0] >= floor * taper.max()
    err = np.linalg.norm((st[0] - want[0])[:, keep]) / np.linalg.norm(want[0, 0][keep])
    print(f"  corrected vs point-kernel image: {err:.3e}")
    assert err <= 1e-4


def test_postprocess_refusals():
    import torch
    from paper_1904_11422_amd import EpicError, Imager
    im = Imager(32, 1, 2, 8)
    img = torch.zeros(im.image_shape(), dtype=torch.complex128, device="cuda")
    with pytest.raises(EpicError, match="STATE"):
        im.postprocess(img)
    inp = synth.random_problem(731, 32, 8, 1, 2, 2)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    with pytest.raises(EpicError, match="INVALID"):
        im.postprocess(img, 1.5)
