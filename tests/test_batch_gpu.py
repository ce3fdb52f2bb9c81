"""Heterogeneous batch (grids of 32^2, 64^2, 128^2; 64, 256 and 1024
antennas) advanced together: every block against the FP64 oracle, HIP graph
replays against the eager batch, and the autotuner's cache."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

# the heterogeneous shapes of the batched workload, fewer channels
BLOCKS = ((32, 64, 12), (32, 64, 3), (64, 256, 6), (64, 256, 2), (128, 1024, 3), (128, 1024, 1))
T = 24


@pytest.fixture(scope="module")
def batch_inputs():
    return [synth.config4_block(b, n_time=T, blocks=BLOCKS) for b in range(len(BLOCKS))]


def _batch(inputs):
    import torch
    from paper_1904_11422_amd import Batch
    cfgs = [dict(grid_n=i.grid_n, n_chan=i.n_chan, n_pol=i.n_pol, n_ant=i.n_ant) for i in inputs]
    b = Batch(cfgs)
    for k, i in enumerate(inputs):
        b.set_antennas(k, i.xy_m, i.freq_hz)
    ef = [torch.from_numpy(np.ascontiguousarray(i.efield)).cuda() for i in inputs]
    g = [torch.from_numpy(np.ascontiguousarray(i.gains)).cuda() for i in inputs]
    return b, ef, g


def test_batch_matches_oracle(batch_inputs):
    import torch
    b, ef, g = _batch(batch_inputs)
    imgs = b.accumulate(ef, g, b.new_images())
    torch.cuda.synchronize()
    for k, inp in enumerate(batch_inputs):
        print(f"block {k}: N={inp.grid_n} A={inp.n_ant} C={inp.n_chan}", flush=True)
        err = oracle.rel_errors(imgs[k].cpu().numpy(), oracle.image_from(inp))
        assert err.max() <= 1e-5, f"block {k}: {err.max():.3e}"


@pytest.mark.parametrize("serial", [False, True])
def test_graph_replays_match_eager(batch_inputs, serial):
    import torch
    b, ef, g = _batch(batch_inputs)
    b.serial = serial
    assert b.serial is serial
    eager = [x.clone() for x in b.accumulate(ef, g, b.new_images())]
    torch.cuda.synchronize()
    out = b.new_images()
    b.capture(ef, g, out)
    for rep in range(3):
        for x in out:
            x.fill_(float("nan"))
        b.replay()
        torch.cuda.synchronize()
        for k in range(len(out)):
            assert torch.equal(out[k], eager[k]), f"replay {rep}, block {k}"
        # eager work of the program between replays
        scratch = b.accumulate(ef, g, b.new_images())
        torch.cuda.synchronize()
        assert torch.equal(scratch[0], eager[0])


def test_tune_then_cache(batch_inputs, tmp_path):
    import torch
    cache = str(tmp_path / "plans.txt")
    b, ef, g = _batch(batch_inputs)
    imgs = b.new_images()
    assert b.tune(ef, g, imgs, cache) is True
    plan = b.plan()
    b2, ef2, g2 = _batch(batch_inputs)
    assert b2.tune(ef2, g2, b2.new_images(), cache) is False
    assert b2.plan() == plan
    for (grid, tb), inp in zip(plan, batch_inputs):
        assert grid > 0 and tb == 0          # every block (two polarisations) runs fused
    out = b2.accumulate(ef2, g2, b2.new_images())
    torch.cuda.synchronize()
    for k, inp in enumerate(batch_inputs):
        err = oracle.rel_errors(out[k].cpu().numpy(), oracle.image_from(inp))
        assert err.max() <= 1e-5


@pytest.mark.slow
def test_full_batch_sampled_channels():
    """The benchmark's batch (six blocks at their full channel counts, T = 200)
    in the launch configuration bench.py times -- tuned plan, captured graph,
    replayed -- checked on two sampled channels of every block against the
    oracle over all 200 samples."""
    import torch
    inputs = [synth.config4_block(b) for b in range(len(synth.CONFIG4_BLOCKS))]
    b, ef, g = _batch(inputs)
    imgs = b.new_images()
    b.tune(ef, g, imgs)
    b.capture(ef, g, imgs)
    b.replay()
    torch.cuda.synchronize()
    for k, inp in enumerate(inputs):
        for c in (0, inp.n_chan - 1):
            print(f"block {k}: N={inp.grid_n} A={inp.n_ant} channel {c}", flush=True)
            sub = synth.Inputs(inp.grid_n, 1, inp.n_pol, inp.n_ant, 3, 0.5, 0.5, inp.xy_m,
                               inp.freq_hz[c:c + 1], inp.gains[c:c + 1], inp.efield[:, c:c + 1])
            err = oracle.rel_errors(imgs[k][c:c + 1].cpu().numpy(), oracle.image_from(sub))
            assert err.max() <= 1e-5, f"block {k} channel {c}: {err.max():.3e}"
