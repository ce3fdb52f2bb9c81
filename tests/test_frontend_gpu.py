"""Front end (decimation + transposition) and the double-buffered streaming
ingest against the oracle.  The front end moves bytes: bit-exact.  Images
after the pipeline: the float32 path's bar, 1e-5 relative per (channel, product)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


def _imager(inp, **kw):
    from paper_1904_11422_amd import Imager
    im = Imager(inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                inp.kernel_sigma_cells, inp.cell_wavelengths, **kw)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    return im


@pytest.mark.parametrize("A,P,c_in,c0,c_step,C,T", [
    (256, 2, 9, 3, 1, 5, 7),      # 16-byte path
    (150, 2, 8, 1, 2, 4, 5),      # byte path (A % 8 != 0)
    (64, 1, 6, 0, 3, 2, 9),       # one polarisation, 8-byte path
    (7, 1, 3, 2, 1, 1, 4),        # one polarisation, bytes
    (16, 2, 4, 0, 1, 4, 1),       # no decimation, one sample
])
def test_frontend_is_bit_exact(A, P, c_in, c0, c_step, C, T):
    import torch
    from paper_1904_11422_amd import Imager
    print(f"case A={A} P={P} c_in={c_in} c0={c0} step={c_step} C={C} T={T}", flush=True)
    raw = synth.raw_gulp(500 + A, T, c_in, A, P)
    im = Imager(32, C, P, A)
    got = im.frontend(torch.from_numpy(raw).cuda(), c0, c_step).cpu().numpy()
    assert np.array_equal(got, oracle.decimate_transpose(raw, C, c0, c_step))


def test_frontend_misaligned_input_takes_the_byte_path():
    import torch
    from paper_1904_11422_amd import Imager
    raw = synth.raw_gulp(510, 3, 5, 64, 2)
    buf = torch.empty(raw.size + 1, dtype=torch.uint8, device="cuda")
    buf[1:] = torch.from_numpy(raw.reshape(-1)).cuda()
    r = buf[1:].view(raw.shape)
    assert r.data_ptr() % 16 != 0
    got = Imager(32, 2, 2, 64).frontend(r, 1, 2).cpu().numpy()
    assert np.array_equal(got, oracle.decimate_transpose(raw, 2, 1, 2))


def test_frontend_rejects_selection_outside_input_and_leaves_output():
    import torch
    from paper_1904_11422_amd import EpicError, Imager
    im = Imager(32, 3, 2, 16)
    raw = torch.from_numpy(synth.raw_gulp(511, 2, 5, 16, 2)).cuda()
    out = torch.full((2, 3, 2, 16), 9, dtype=torch.uint8, device="cuda")
    for c0, step in [(3, 1), (0, 3), (-1, 1), (0, 0)]:
        with pytest.raises(EpicError, match="INVALID"):
            im.frontend(raw, c0, step, out=out)
    torch.cuda.synchronize()
    assert torch.all(out == 9)


def _gulps(seed, n, T, c_in, A, P):
    import torch
    out = []
    for k in range(n):
        g = torch.from_numpy(synth.raw_gulp(seed + k, T, c_in, A, P)).pin_memory()
        out.append(g)
    return out


@pytest.mark.parametrize("c0,c_step,remove_autos", [(2, 1, False), (1, 2, False), (0, 3, True)])
def test_pipeline_images_every_gulp(c0, c_step, remove_autos):
    """Gulps of different data pushed back to back (the copy of one overlapping
    the imaging of the one before): the accumulated image equals the oracle's
    sum over the gulps of the decimated, transposed data."""
    import torch
    from paper_1904_11422_amd import Pipeline
    base = synth.random_problem(520, 32, 24, 3, 2, 1)
    T, c_in, n = 11, 10, 6
    print(f"case c0={c0} step={c_step} autos={remove_autos}", flush=True)
    im = _imager(base, remove_autos=remove_autos)
    pipe = Pipeline(im, T, c_in, c0, c_step)
    g = torch.from_numpy(base.gains).cuda()
    img = torch.empty(im.image_shape(), dtype=torch.complex128, device="cuda")
    gulps = _gulps(530, n, T, c_in, 24, 2)
    for k, h in enumerate(gulps):
        pipe.push(h, g, img, reset=(k == 0))
    st = pipe.report()
    assert st["gulps"] == n
    ef = np.concatenate([oracle.decimate_transpose(h.numpy(), 3, c0, c_step) for h in gulps])
    fn = oracle.image_without_autos if remove_autos else oracle.image
    ref = fn(base.xy_m, base.freq_hz, base.gains, ef, 32)
    full = oracle.image(base.xy_m, base.freq_hz, base.gains, ef, 32)
    got = img.cpu().numpy()
    d = np.linalg.norm((got - ref).reshape(3, 4, -1), axis=-1)
    r = np.linalg.norm(full.reshape(3, 4, -1), axis=-1)
    r[:, 1] = r[:, 2] = np.sqrt(r[:, 0] * r[:, 3])
    assert np.max(d / r) <= TOL_FP32, f"{np.max(d / r):.3e}"
    pipe.close()


def test_pipeline_one_image_per_gulp_and_ring_wrap():
    """More gulps than the ring holds (64), each into its own image: every image
    matches its gulp, and every gulp is counted."""
    import torch
    from paper_1904_11422_amd import Pipeline
    base = synth.random_problem(540, 32, 16, 1, 1, 1)
    T, c_in, n = 3, 2, 70
    im = _imager(base)
    pipe = Pipeline(im, T, c_in, 1, 1)
    g = torch.from_numpy(base.gains).cuda()
    gulps = _gulps(550, n, T, c_in, 16, 1)
    imgs = [torch.empty(im.image_shape(), dtype=torch.complex128, device="cuda") for _ in range(n)]
    for h, out in zip(gulps, imgs):
        pipe.push(h, g, out)
    st = pipe.report()
    assert st["gulps"] == n
    for k in (0, 31, 63, 64, 69):
        ef = oracle.decimate_transpose(gulps[k].numpy(), 1, 1, 1)
        ref = oracle.image(base.xy_m, base.freq_hz, base.gains, ef, 32)
        assert oracle.rel_errors(imgs[k].cpu().numpy(), ref).max() <= TOL_FP32, k


@pytest.mark.parametrize("sample_s,expect_all", [(1e-12, True), (10.0, False)])
def test_pipeline_real_time_check(sample_s, expect_all):
    """Budget check forced from the host: a gulp that spans almost no time is
    always over budget, one that spans hours never is."""
    import torch
    from paper_1904_11422_amd import Pipeline
    base = synth.random_problem(560, 32, 16, 2, 2, 1)
    im = _imager(base)
    pipe = Pipeline(im, 4, 2, 0, 1, sample_s=sample_s)
    g = torch.from_numpy(base.gains).cuda()
    img = torch.empty(im.image_shape(), dtype=torch.complex128, device="cuda")
    for h in _gulps(570, 5, 4, 2, 16, 2):
        pipe.push(h, g, img)
    st = pipe.report()
    assert st["gulps"] == 5
    assert st["over_budget"] == (5 if expect_all else 0)
    assert st["mean_ms"] > 0 and st["max_ms"] >= st["mean_ms"]
    assert abs(st["gulp_ms"] - 4 * sample_s * 1e3) <= 1e-9 * max(1.0, st["gulp_ms"])


def test_pipeline_errors():
    import torch
    from paper_1904_11422_amd import EpicError, Imager, Pipeline, _lib
    im = Imager(32, 2, 2, 16)
    with pytest.raises(EpicError, match="INVALID"):
        Pipeline(im, 4, 2, 1, 1)                  # channel 2 outside c_in = 2
    with pytest.raises(EpicError, match="INVALID"):
        Pipeline(im, 0, 2, 0, 1)
    pipe = Pipeline(im, 4, 2, 0, 1)
    h = _gulps(580, 1, 4, 2, 16, 2)[0]
    g = torch.ones((2, 2, 16), dtype=torch.complex64, device="cuda")
    img = torch.empty(im.image_shape(), dtype=torch.complex128, device="cuda")
    with pytest.raises(EpicError, match="STATE"):
        pipe.push(h, g, img)                      # no antennas yet
    st = _lib.PipelineStats()
    assert im.L.epic_pipeline_report(pipe._p, ctypes.byref(st)) == 0
    assert st.gulps == 0
    pipe.close()
