"""Seeded sweep over the configuration space against the FP64 oracle: grid
size, polarisations, antenna and channel counts, sample counts, kernel
support, the caller's complex kernels, apertures wider than N/2 (the wide
fused variant at N = 64 up to 48 cells, else the staged route), the staged flag and autocorrelation removal, each through the image
and through the gain gradient; and the split forms within their antenna
limits.  Each case is drawn from its own seed, so a failure names a
reproducible configuration.

Bars as in the targeted tests: images 1e-5 relative per (channel, product)
(float32 paths; removed images against the full image's norm), 1e-3 (split
forms), gradients 1e-4 relative L2."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_SPLIT = 1e-3
TOL_GRAD = 1e-4


def _draw(seed):
    """One configuration of the float32 paths."""
    rng = np.random.default_rng(seed)
    N = int(rng.choice([32, 64, 128], p=[0.4, 0.4, 0.2]))
    P = int(rng.integers(1, 3))
    wide = rng.random() < 0.2                      # aperture wider than N/2: wide fused or staged
    fill = float(rng.uniform(0.55, 0.7) if wide else rng.uniform(0.25, 0.45))
    # antennas the seeded disk can hold at half-cell separation
    room = int(0.3 * ((fill * N - 3) / 0.5) ** 2)
    a_max = min({32: 120, 64: 400, 128: 1100}[N], max(1, room))
    A = int(rng.integers(1, a_max + 1))
    C = int(rng.integers(1, 4))
    T = int(rng.integers(1, 24 if N < 128 else 8))
    K = int(rng.choice([3, 3, 3, 5, 7]))
    cplx = K != 3 or rng.random() < 0.25
    staged = bool(rng.random() < 0.15)
    autos = bool(rng.random() < 0.3)
    return dict(N=N, P=P, A=A, C=C, T=T, fill=fill, K=K, cplx=cplx, staged=staged, autos=autos)


def _case(seed):
    d = _draw(seed)
    inp = synth.random_problem(seed, d["N"], d["A"], d["C"], d["P"], d["T"], fill=d["fill"])
    if d["cplx"]:
        inp = synth.with_kernels(inp, d["K"], seed + 7)
    return d, inp


def _norms(full, n_chan, n_pol):
    """Per (channel, product) reference norms; XY and YX against sqrt(|XX| |YY|).
    A product that is exactly zero in the reference (a polarisation whose few
    samples are all zero) is measured against the channel's largest norm."""
    nrm = np.linalg.norm(full.reshape(n_chan, full.shape[1], -1), axis=-1)
    if n_pol == 2:
        nrm[:, 1] = nrm[:, 2] = np.sqrt(nrm[:, 0] * nrm[:, 3])
    top = np.maximum(nrm.max(axis=1, keepdims=True), np.finfo(float).tiny)
    return np.where(nrm > 0, nrm, top)


@pytest.mark.parametrize("seed", range(5000, 5032))
def test_fp32_image_and_gradient(seed):
    import torch
    from paper_1904_11422_amd import Imager
    d, inp = _case(seed)
    print(f"seed {seed}: {d}", flush=True)
    im = Imager(inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                inp.kernel_sigma_cells, inp.cell_wavelengths, staged=d["staged"],
                remove_autos=d["autos"])
    im.set_antennas(inp.xy_m, inp.freq_hz, kernels=inp.kernels)
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    got = im.accumulate(ef, g).cpu().numpy()
    full = oracle.image_from(inp)
    ref = oracle.image_without_autos_from(inp) if d["autos"] else full
    nrm = _norms(full, inp.n_chan, inp.n_pol)
    err = np.linalg.norm((got - ref).reshape(inp.n_chan, got.shape[1], -1), axis=-1) / nrm
    print(f"  route {im.last_kernel_name()}, image err {err.max():.3e}", flush=True)
    assert np.all(np.isfinite(got))
    assert err.max() <= TOL_FP32, f"{err.max():.3e}"
    # gain gradient of an L2 loss on that image
    rng = np.random.default_rng(seed)
    gam = oracle.l2_loss_grad_image(got, got * (1 + 0.05 * rng.normal(size=got.shape)))
    gg = im.backward(ef, g, torch.from_numpy(gam).cuda()).cpu().numpy()
    fn = oracle.grad_gains_without_autos if d["autos"] else oracle.grad_gains
    gref = fn(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, inp.grid_n, gam, inp.kernel_support,
              kernels=inp.kernels)
    gerr = np.linalg.norm(gg - gref) / np.linalg.norm(gref)
    print(f"  gradient err {gerr:.3e}", flush=True)
    assert gerr <= TOL_GRAD, f"{gerr:.3e}"


@pytest.mark.parametrize("seed", range(5100, 5112))
def test_split_forms(seed):
    import torch
    from paper_1904_11422_amd import Imager
    rng = np.random.default_rng(seed)
    N = int(rng.choice([32, 64]))
    P = int(rng.integers(1, 3))
    A = int(rng.integers(1, (32 if P == 1 else 16) + 1))
    C = int(rng.integers(1, 4))
    T = int(rng.integers(1, 700))
    prec = str(rng.choice(["split_fp16", "split_bf16"]))
    autos = bool(rng.random() < 0.3)
    inp = synth.random_problem(seed, N, A, C, P, T, fill=float(rng.uniform(0.3, 0.45)))
    print(f"seed {seed}: N={N} P={P} A={A} C={C} T={T} {prec} autos={autos}", flush=True)
    im = Imager(N, C, P, A, precision=prec, remove_autos=autos)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    got = im.accumulate(ef, g).cpu().numpy()
    assert im.last_kernel_name() == "split_image_kernel"
    full = oracle.image_from(inp)
    ref = oracle.image_without_autos_from(inp) if autos else full
    nrm = _norms(full, C, P)
    err = np.linalg.norm((got - ref).reshape(C, got.shape[1], -1), axis=-1) / nrm
    print(f"  image err {err.max():.3e}", flush=True)
    assert err.max() <= TOL_SPLIT, f"{err.max():.3e}"


@pytest.mark.parametrize("seed", range(5200, 5210))
def test_wide_block_image_and_gradient(seed):
    """Apertures of 33-48 cells at N = 64 (the wide fused kernel and its
    adjoint): random polarisations, antenna and channel counts, samples, kernel
    support (Gaussian or the caller's complex kernels) and autocorrelation
    removal."""
    import torch
    from paper_1904_11422_amd import Imager
    rng = np.random.default_rng(seed)
    P = int(rng.integers(1, 3))
    K = int(rng.choice([3, 3, 5, 7]))
    fill = float(rng.uniform(0.55, 0.74 - (K - 3) / 64))
    A = int(rng.integers(2, 500))
    C = int(rng.integers(1, 4))
    T = int(rng.integers(1, 16))
    autos = bool(rng.random() < 0.3) and K <= 7
    inp = synth.random_problem(seed, 64, A, C, P, T, fill=fill)
    # two antennas at opposite ends of the disk's east-west diameter: the
    # aperture spans fill * 64 - 3 > 32 cells at every channel, so the case
    # always takes the wide block whatever the draw
    radius = 0.5 * (fill * 64 - 3) * 0.5 * synth.C0 / inp.freq_hz.max()
    inp.xy_m[0] = (radius, 0.0)
    inp.xy_m[1] = (-radius, 0.0)
    if K != 3 or rng.random() < 0.3:
        inp = synth.with_kernels(inp, K, seed + 7)
    print(f"seed {seed}: P={P} A={A} C={C} T={T} K={K} fill={fill:.3f} autos={autos}", flush=True)
    im = Imager(64, C, P, A, inp.kernel_support, remove_autos=autos)
    im.set_antennas(inp.xy_m, inp.freq_hz, kernels=inp.kernels)
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    got = im.accumulate(ef, g).cpu().numpy()
    kname = im.last_kernel_name()
    print(f"  route {kname}", flush=True)
    assert kname == "fused_wide_image_kernel"
    full = oracle.image_from(inp)
    ref = oracle.image_without_autos_from(inp) if autos else full
    err = np.linalg.norm((got - ref).reshape(C, got.shape[1], -1), axis=-1) / _norms(full, C, P)
    assert err.max() <= TOL_FP32, f"{err.max():.3e}"
    gam = oracle.l2_loss_grad_image(got, got * (1 + 0.05 * rng.normal(size=got.shape)))
    gg = im.backward(ef, g, torch.from_numpy(gam).cuda()).cpu().numpy()
    fn = oracle.grad_gains_without_autos if autos else oracle.grad_gains
    gref = fn(inp.xy_m, inp.freq_hz, inp.gains, inp.efield, 64, gam, inp.kernel_support,
              kernels=inp.kernels)
    gerr = np.linalg.norm(gg - gref) / np.linalg.norm(gref)
    print(f"  image err {err.max():.3e}, gradient err {gerr:.3e}", flush=True)
    assert gerr <= TOL_GRAD, f"{gerr:.3e}"
