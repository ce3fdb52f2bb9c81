"""Split-precision (float16 / bfloat16 hi+lo) MFMA form of gridding + transform
against the FP64 oracle.  Bar: relative L2 error per (channel, product)
<= 1e-3; float16 hi+lo carries ~2^-22 relative per matrix entry,
bfloat16 hi+lo ~2^-16, the products are summed in float64."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_SPLIT = 1e-3


def _run(inp, precision, reset_split=None):
    import torch
    from paper_1904_11422_amd import Imager
    print(f"case {inp.name}: N={inp.grid_n} C={inp.n_chan} P={inp.n_pol} A={inp.n_ant} "
          f"T={inp.n_time} {precision}", flush=True)
    im = Imager(inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                inp.kernel_sigma_cells, inp.cell_wavelengths, precision=precision)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    ef = torch.from_numpy(np.ascontiguousarray(inp.efield)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(inp.gains)).cuda()
    if reset_split is None:
        out = im.accumulate(ef, g)
    else:
        out = im.accumulate(ef[:reset_split], g)
        im.accumulate(ef[reset_split:], g, image=out, reset=False)
    torch.cuda.synchronize()
    assert im.last_kernel_name() == "split_image_kernel"
    return out.cpu().numpy()


CASES = {
    "cfg1": lambda: synth.config1(),
    "cfg3_t2000": lambda: synth.config3(n_time=2000),
    "p2_a16": lambda: synth.random_problem(301, 32, 16, 2, 2, 45),
    "p1_a32_n64": lambda: synth.random_problem(302, 64, 32, 2, 1, 70),
    "p1_a7_ragged": lambda: synth.random_problem(303, 32, 7, 3, 1, 33),
    # chunks of 9 blocks (not a multiple of the 4-block sample ring), a
    # 16-sample last chunk
    "cfg3_t70000": lambda: synth.config3(n_time=70_000),
    # two polarisations over 12 chunks of 256 samples (2-block ring), the last
    # one 184 samples long
    "p2_a16_t3000": lambda: synth.random_problem(305, 32, 16, 1, 2, 3000),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["split_fp16", "split_bf16"])
def test_split_matches_oracle(name, precision):
    inp = CASES[name]()
    got = _run(inp, precision)
    ref = oracle.image_from(inp)
    err = oracle.rel_errors(got, ref)
    print(f"  max rel err {err.max():.3e}")
    assert np.all(np.isfinite(got))
    assert err.max() <= TOL_SPLIT, f"{err.max():.3e}"


def test_split_fp16_is_tighter_than_bf16():
    inp = synth.config3(n_time=4000)
    ref = oracle.image_from(inp)
    e16 = oracle.rel_errors(_run(inp, "split_fp16"), ref).max()
    e_bf = oracle.rel_errors(_run(inp, "split_bf16"), ref).max()
    print(f"fp16 {e16:.2e} bf16 {e_bf:.2e}")
    assert e16 < 1e-5 and e_bf < TOL_SPLIT and e16 < e_bf


def test_split_reset_continuation():
    inp = synth.random_problem(304, 32, 16, 1, 2, 70)
    got = _run(inp, "split_fp16", reset_split=33)
    assert oracle.rel_errors(got, oracle.image_from(inp)).max() <= TOL_SPLIT


def test_split_rejects_large_arrays():
    from paper_1904_11422_amd import EpicError, Imager
    with pytest.raises(EpicError, match="UNSUPPORTED"):
        Imager(64, 4, 2, 256, precision="split_fp16")


@pytest.mark.slow
def test_config3_full_integration():
    """10^5 samples of the tiny geometry, both split forms, float64 long sums."""
    inp = synth.config3()
    ref = oracle.image_from(inp)
    for prec in ("split_fp16", "split_bf16"):
        err = oracle.rel_errors(_run(inp, prec), ref).max()
        print(f"{prec}: {err:.3e}")
        assert err <= TOL_SPLIT
