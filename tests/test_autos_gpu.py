"""Autocorrelation removal (EPIC_FLAG_REMOVE_AUTOS) against the FP64 oracle.

Tolerances.  The removal itself is exact integer sums plus float64 arithmetic
on the library's float32 kernel weights, so the removed term (the difference
between a call without and a call with the flag, whose full images are
bit-identical) matches the oracle's float64-weight autocorrelation image to
the weights' rounding: each R_a(d) is a sum of products of two float32-rounded
weights, relative error <= ~2^-23, bar 1e-6 of the autocorrelation image's
norm.  The removed image carries the float32 imaging error of the full image,
so its bar is the float32 path's 1e-5, taken relative to the full image's
norm (XY, YX: to sqrt(|XX| |YY|) of the full image)."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_AUTOS = 1e-6
TOL_GRAD = 1e-4


def _imager(inp, remove_autos=True, staged=False, precision="fp32", timing=False):
    from paper_1904_11422_amd import Imager
    im = Imager(inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                inp.kernel_sigma_cells, inp.cell_wavelengths, precision=precision,
                staged=staged, timing=timing, remove_autos=remove_autos)
    im.set_antennas(inp.xy_m, inp.freq_hz, kernels=inp.kernels)
    return im


def _cplx(seed, N, A, C, P, T, K, fill=0.4):
    return synth.with_kernels(synth.random_problem(seed, N, A, C, P, T, fill=fill), K, seed + 1)


def _dev(inp):
    import torch
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    return ef, g


def _errors(got, ref, full):
    """Per (channel, product) L2 error of got vs ref, relative to the norm of
    the full image (XY, YX: sqrt of the XX and YY norms)."""
    d = np.linalg.norm((got - ref).reshape(got.shape[0], got.shape[1], -1), axis=-1)
    r = np.linalg.norm(full.reshape(full.shape[0], full.shape[1], -1), axis=-1)
    if got.shape[1] == 4:
        sx = np.sqrt(r[:, 0] * r[:, 3])
        r = np.stack([r[:, 0], sx, sx, r[:, 3]], axis=1)
    return d / np.maximum(r, 1e-300)


def _run_both(inp, **kw):
    import torch
    print(f"case {inp.name}: N={inp.grid_n} C={inp.n_chan} P={inp.n_pol} A={inp.n_ant} "
          f"K={inp.kernel_support} T={inp.n_time} {kw}", flush=True)
    ef, g = _dev(inp)
    full = _imager(inp, remove_autos=False, **kw).accumulate(ef, g)
    im = _imager(inp, remove_autos=True, **kw)
    removed = im.accumulate(ef, g)
    torch.cuda.synchronize()
    return full.cpu().numpy(), removed.cpu().numpy(), im


def _k5(seed, grid_n, n_ant, n_chan, n_pol, n_time):
    inp = synth.random_problem(seed, grid_n, n_ant, n_chan, n_pol, n_time, fill=0.4)
    return dataclasses.replace(inp, kernel_support=5, kernel_sigma_cells=0.9,
                               name=f"{inp.name}_k5")


CASES = {
    # (inputs, imager options)
    "n32_p2_ragged": (lambda: synth.random_problem(401, 32, 64, 3, 2, 37), {}),
    "n64_p1": (lambda: synth.random_problem(402, 64, 100, 2, 1, 10), {}),
    "n64_p2_A150_bytes": (lambda: synth.random_problem(403, 64, 150, 2, 2, 11, fill=0.45), {}),
    "n64_p2_k5": (lambda: _k5(404, 64, 96, 2, 2, 13), {}),
    "n128_p2": (lambda: synth.random_problem(405, 128, 400, 2, 2, 5, fill=0.45), {}),
    "n64_p2_staged": (lambda: synth.random_problem(406, 64, 64, 2, 2, 9), {"staged": True}),
    "n64_p2_wide": (lambda: synth.random_problem(410, 64, 140, 2, 2, 9, fill=0.66), {}),
    "n128_p1": (lambda: synth.random_problem(407, 128, 200, 1, 1, 4, fill=0.45), {}),
    "n128_p1_staged": (lambda: synth.random_problem(407, 128, 200, 1, 1, 4, fill=0.45),
                       {"staged": True}),
    "split16_p2": (lambda: synth.random_problem(408, 32, 16, 2, 2, 45),
                   {"precision": "split_fp16"}),
    "split_bf16_p1_A7": (lambda: synth.random_problem(409, 32, 7, 3, 1, 33),
                         {"precision": "split_bf16"}),
    "cfg1": (lambda: synth.config1(), {}),
    # the caller's complex kernels
    "n64_p2_k5_complex": (lambda: _cplx(441, 64, 96, 2, 2, 9, 5), {}),
    "n32_p1_k3_complex": (lambda: _cplx(442, 32, 36, 2, 1, 11, 3), {}),
    "n128_p2_k7_complex": (lambda: _cplx(443, 128, 200, 2, 2, 4, 7, fill=0.4), {}),
    "n64_p2_k3_complex_staged": (lambda: _cplx(444, 64, 50, 2, 2, 6, 3), {"staged": True}),
    "split16_p2_k5_complex": (lambda: _cplx(445, 32, 16, 2, 2, 30, 5), {"precision": "split_fp16"}),
}


@pytest.mark.parametrize("name", list(CASES))
def test_removed_image_matches_oracle(name):
    make, kw = CASES[name]
    inp = make()
    full, got, _ = _run_both(inp, **kw)
    ref = oracle.image_without_autos_from(inp)
    ref_full = oracle.image_from(inp)
    autos = oracle.autocorrelation_image(inp.xy_m, inp.freq_hz, inp.gains, inp.efield,
                                         inp.grid_n, inp.kernel_support, inp.kernel_sigma_cells,
                                         inp.cell_wavelengths, inp.kernels)
    assert np.all(np.isfinite(got))
    # the removed term alone, to the weights' rounding
    dr = np.linalg.norm((full - got - autos).reshape(inp.n_chan, -1), axis=-1)
    na = np.linalg.norm(autos.reshape(inp.n_chan, -1), axis=-1)
    assert np.all(dr <= TOL_AUTOS * na), f"removed term err {np.max(dr / na):.3e}"
    # the image without autocorrelations, to the float32 imaging bar
    tol = 1e-3 if "split" in name else TOL_FP32
    err = _errors(got, ref, ref_full)
    print(f"  max err {err.max():.3e} (removed term {np.max(dr / na):.3e})")
    assert err.max() <= tol, f"{err.max():.3e}"
    if inp.n_pol == 2:
        assert np.array_equal(got[:, 2], np.conj(got[:, 1]))
        assert np.array_equal(got[:, 0].imag, full[:, 0].imag)


def test_single_antenna_leaves_float32_noise_only():
    """One antenna: the whole image is its autocorrelation (closed form)."""
    inp = synth.random_problem(410, 64, 1, 2, 2, 25)
    full, got, _ = _run_both(inp)
    for p in range(got.shape[1]):
        assert np.linalg.norm(got[:, p]) <= TOL_FP32 * np.linalg.norm(full[:, 0]), p


def test_split_integration_adds_up():
    """Removal per call is linear in the samples: two calls with reset=0 equal
    the oracle over all samples."""
    import torch
    inp = synth.random_problem(411, 32, 48, 2, 2, 30)
    im = _imager(inp)
    ef, g = _dev(inp)
    out = im.accumulate(ef[:13], g)
    im.accumulate(ef[13:], g, image=out, reset=False)
    torch.cuda.synchronize()
    err = _errors(out.cpu().numpy(), oracle.image_without_autos_from(inp), oracle.image_from(inp))
    assert err.max() <= TOL_FP32, f"{err.max():.3e}"


def test_unaligned_efield_takes_the_byte_path():
    """A 4-byte misaligned E-field (A % 4 == 0) is read one byte at a time."""
    import torch
    inp = synth.random_problem(412, 32, 32, 2, 2, 21)
    im = _imager(inp)
    raw = np.ascontiguousarray(inp.efield).reshape(-1)
    buf = torch.empty(raw.size + 1, dtype=torch.uint8, device="cuda")
    buf[1:] = torch.from_numpy(raw).cuda()
    ef = buf[1:].view(inp.efield.shape)
    assert ef.data_ptr() % 4 != 0
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    got = im.accumulate(ef, g).cpu().numpy()
    err = _errors(got, oracle.image_without_autos_from(inp), oracle.image_from(inp))
    assert err.max() <= TOL_FP32, f"{err.max():.3e}"


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("seed,N,A,C,P,T,K", [(421, 32, 16, 2, 2, 5, 0), (422, 32, 20, 1, 1, 7, 0),
                                            (423, 64, 256, 3, 2, 11, 0), (424, 64, 90, 2, 1, 4, 0),
                                            (425, 64, 150, 2, 2, 6, 0), (426, 32, 24, 2, 2, 5, 5),
                                            (427, 64, 80, 2, 1, 4, 3), (429, 128, 300, 2, 2, 3, 0),
                                            (430, 128, 200, 1, 1, 4, 5)])
def test_grad_without_autos_matches_oracle(seed, N, A, C, P, T, K):
    """Gain gradient of an L2 loss on the removed image (bar of the gradient:
    1e-4 relative); the removed term's share (full-image gradient minus this
    one, both float32-rounded from identical float64 sums) to 1e-6 of the
    full gradient."""
    import torch
    inp = _cplx(seed, N, A, C, P, T, K, fill=0.35) if K else synth.random_problem(seed, N, A, C, P, T)
    print(f"case {inp.name}: N={N} C={C} P={P} A={A} T={T} K={inp.kernel_support}", flush=True)
    ef, g = _dev(inp)
    im = _imager(inp)
    img = im.accumulate(ef, g).cpu().numpy()
    rng = np.random.default_rng(seed)
    model = img * (1 + 0.05 * rng.normal(size=img.shape)) + rng.normal(size=img.shape)
    gam = oracle.l2_loss_grad_image(img, model)
    gam_d = torch.from_numpy(gam).cuda()
    got = im.backward(ef, g, gam_d).cpu().numpy()
    Kk = inp.kernel_support
    ref = oracle.grad_gains_without_autos(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, N, gam, Kk,
                                          kernels=inp.kernels)
    assert _rel(got, ref) <= TOL_GRAD, f"{_rel(got, ref):.3e}"
    full = _imager(inp, remove_autos=False).backward(ef, g, gam_d).cpu().numpy()
    share = oracle.grad_autos(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, N, gam, Kk,
                              kernels=inp.kernels)
    d = np.linalg.norm((full - got) - share) / np.linalg.norm(full)
    print(f"  grad err {_rel(got, ref):.3e}, share err {d:.3e}")
    assert d <= TOL_AUTOS, f"{d:.3e}"


@pytest.mark.parametrize("P", [1, 2])
def test_grad_without_autos_on_staged_kernels(P):
    """The staged gradient with the autocorrelation terms removed."""
    import torch
    inp = synth.random_problem(431 + P, 32, 30, 2, P, 6)
    ef, g = _dev(inp)
    im = _imager(inp, staged=True)
    img = im.accumulate(ef, g).cpu().numpy()
    rng = np.random.default_rng(431)
    model = img * (1 + 0.05 * rng.normal(size=img.shape)) + rng.normal(size=img.shape)
    gam = oracle.l2_loss_grad_image(img, model)
    got = im.backward(ef, g, torch.from_numpy(gam).cuda()).cpu().numpy()
    assert im.last_kernel_name() == "staged_degrid_kernel"
    ref = oracle.grad_gains_without_autos(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 32, gam)
    assert _rel(got, ref) <= TOL_GRAD, f"{_rel(got, ref):.3e}"


def test_grad_single_antenna_vanishes():
    import torch
    inp = synth.random_problem(426, 32, 1, 2, 2, 9)
    ef, g = _dev(inp)
    rng = np.random.default_rng(4)
    gam = torch.from_numpy(rng.normal(size=(2, 4, 32, 32)) + 1j * rng.normal(size=(2, 4, 32, 32))).cuda()
    got = _imager(inp).backward(ef, g, gam).cpu().numpy()
    full = _imager(inp, remove_autos=False).backward(ef, g, gam).cpu().numpy()
    assert np.linalg.norm(got) <= TOL_GRAD * np.linalg.norm(full)


def test_autograd_without_autos():
    """torch.autograd through image() of an imager with remove_autos."""
    import torch
    from paper_1904_11422_amd import image
    inp = synth.random_problem(427, 32, 24, 2, 2, 8)
    ef, g0 = _dev(inp)
    im = _imager(inp)
    g = g0.clone().requires_grad_(True)
    out = image(im, g, ef)
    w = torch.from_numpy(np.random.default_rng(5).normal(size=out.shape)).cuda()
    loss = (out.real * w).sum()
    loss.backward()
    gam = w.cpu().numpy().astype(complex)
    ref = oracle.grad_gains_without_autos(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 32, gam)
    assert _rel(g.grad.cpu().numpy(), ref) <= TOL_GRAD


def test_limits_and_unsupported_calls_leave_outputs_untouched():
    import torch
    from paper_1904_11422_amd import EpicError
    inp = synth.random_problem(413, 32, 16, 1, 2, 3)
    im = _imager(inp)
    ef, g = _dev(inp)
    out = torch.full(im.image_shape(), 5.0, dtype=torch.complex128, device="cuda")
    from paper_1904_11422_amd import _lib
    import ctypes
    # 2^24 samples: refused before anything is enqueued (efield is never read)
    st = im.L.epic_image_accumulate(im._ctx, ctypes.c_void_p(ef.data_ptr()), 1 << 24,
                                    ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(out.data_ptr()), 1)
    assert st == _lib.EPIC_E_UNSUPPORTED
    gg = torch.zeros_like(g)
    st = im.L.epic_image_backward(im._ctx, ctypes.c_void_p(ef.data_ptr()), 1 << 24,
                                  ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(gg.data_ptr()))
    assert st == _lib.EPIC_E_UNSUPPORTED
    small = synth.random_problem(428, 32, 16, 1, 2, 2)
    ef2, g2 = _dev(small)
    im2 = _imager(small, precision="split_fp16")           # no gradient on the split forms
    with pytest.raises(EpicError, match="UNSUPPORTED"):
        im2.backward(ef2, g2, torch.ones(im2.image_shape(), dtype=torch.complex128, device="cuda"))
    torch.cuda.synchronize()
    assert torch.all(gg == 0)
    assert torch.all(out == 5.0)


def test_timing_reports_the_removal():
    import torch
    inp = synth.random_problem(414, 64, 256, 4, 2, 64)
    im = _imager(inp, timing=True)
    ef, g = _dev(inp)
    im.accumulate(ef, g)
    torch.cuda.synchronize()
    s, r = im.last_autos_timing()
    m, c = im.last_timing()
    assert 0 < s <= r <= c


def test_batch_block_with_removal():
    """A batch block built with remove_autos runs the removal too (graph replay)."""
    import torch
    from paper_1904_11422_amd import Batch
    a = synth.random_problem(415, 32, 64, 2, 2, 17)
    b = synth.random_problem(416, 64, 128, 3, 2, 17)
    cfgs = [dict(a.config_dict(), remove_autos=True), dict(b.config_dict())]
    bt = Batch(cfgs)
    for i, inp in enumerate((a, b)):
        bt.set_antennas(i, inp.xy_m, inp.freq_hz)
    ef = [_dev(x)[0] for x in (a, b)]
    g = [_dev(x)[1] for x in (a, b)]
    imgs = bt.new_images()
    bt.capture(ef, g, imgs)
    refs = [oracle.image_without_autos_from(a), oracle.image_from(b)]
    for _ in range(3):
        for im_ in imgs:
            im_.fill_(9.0)
        bt.replay()
        torch.cuda.synchronize()
        err0 = _errors(imgs[0].cpu().numpy(), refs[0], oracle.image_from(a)).max()
        err1 = oracle.rel_errors(imgs[1].cpu().numpy(), refs[1]).max()
        assert err0 <= TOL_FP32 and err1 <= TOL_FP32, (err0, err1)


@pytest.mark.slow
def test_config2_full_size_sampled_channels_removed():
    """The benchmark's shape (N=64, C=132, P=2, A=256, T=1000) with removal,
    checked on sampled channels against the oracle over all samples."""
    import torch
    inp = synth.config2()
    ef, g = _dev(inp)
    im = _imager(inp)
    got = im.accumulate(ef, g).cpu().numpy()
    torch.cuda.synchronize()
    for c in (0, 77, 131):
        sub = synth.Inputs(inp.grid_n, 1, inp.n_pol, inp.n_ant, 3, 0.5, 0.5, inp.xy_m,
                           inp.freq_hz[c:c + 1], inp.gains[c:c + 1], inp.efield[:, c:c + 1])
        err = _errors(got[c:c + 1], oracle.image_without_autos_from(sub), oracle.image_from(sub))
        assert err.max() <= TOL_FP32, f"channel {c}: {err.max():.3e}"
