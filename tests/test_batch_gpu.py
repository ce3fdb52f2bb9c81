"""Heterogeneous batch (grids of 32^2, 64^2, 128^2; 64, 256 and 1024
antennas) advanced together: every block against the FP64 oracle, HIP graph
replays against the eager batch, the cut into grouped launches (one
persistent launch per grid family walking all its blocks' channels), every
launch shape the autotuner can pick, and the autotuner's cache."""
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


def _check_blocks(imgs, inputs, tol=1e-5):
    for k, inp in enumerate(inputs):
        print(f"block {k}: N={inp.grid_n} A={inp.n_ant} C={inp.n_chan} T={inp.n_time}", flush=True)
        err = oracle.rel_errors(imgs[k].cpu().numpy(), oracle.image_from(inp))
        assert err.max() <= tol, f"block {k}: {err.max():.3e}"


def test_launches_group_blocks_by_grid(batch_inputs):
    """The six blocks form three launches (one per grid side), two blocks each."""
    b, ef, g = _batch(batch_inputs)
    lp = b.launch_plan()
    print(lp, flush=True)
    assert [x[0] for x in lp] == [0, 0, 1, 1, 2, 2]
    assert all(x[1] == 2 for x in lp)


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


def test_mixed_antenna_counts_share_a_launch():
    """Blocks of one grid side with different antenna counts (one sample byte
    per thread) share a launch: workgroups whose range crosses a block boundary
    switch inputs, programs and the E' layout there.  T is ragged so ranges
    start mid-channel; one block has a single channel."""
    import torch
    blocks = ((64, 256, 3), (64, 97, 1), (64, 200, 2), (64, 31, 2))
    inputs = [synth.config4_block(k, n_time=13, blocks=blocks) for k in range(len(blocks))]
    b, ef, g = _batch(inputs)
    lp = b.launch_plan()
    assert [x[0] for x in lp] == [0, 0, 0, 0] and lp[0][1] == 4
    imgs = b.accumulate(ef, g, b.new_images())
    torch.cuda.synchronize()
    _check_blocks(imgs, inputs)
    # continuation: reset = 0 adds the same samples again
    b.accumulate(ef, g, imgs, reset=False)
    torch.cuda.synchronize()
    for k, inp in enumerate(inputs):
        ref = 2.0 * oracle.image_from(inp)
        assert oracle.rel_errors(imgs[k].cpu().numpy(), ref).max() <= 1e-5


def test_many_antenna_blocks_share_a_launch():
    """64^2 blocks of 600, 1000 and 777 dual-pol antennas (four sample bytes
    per thread, E' staged in the second polarisation's upper grid rows) in
    one grouped launch: workgroups that cross a block boundary take the next
    block's antenna count, E' layout and zero slots."""
    import torch
    inputs = [synth.random_problem(821, 64, 600, 3, 2, 9, fill=0.45),
              synth.random_problem(822, 64, 1000, 2, 2, 9, fill=0.48),
              synth.random_problem(823, 64, 777, 1, 2, 9, fill=0.4)]
    b, ef, g = _batch(inputs)
    lp = b.launch_plan()
    print(lp, flush=True)
    assert [x[0] for x in lp] == [0, 0, 0] and lp[0][1] == 3
    imgs = b.accumulate(ef, g, b.new_images())
    torch.cuda.synchronize()
    _check_blocks(imgs, inputs)


def test_wide_blocks_of_both_orientations_share_a_launch():
    """Apertures wider than N/2 at N = 64 in one grouped launch: blocks whose
    wide block has 40 or 48 rows and whose taps are transposed or not (the
    deployed ellipse, elongated along the rows, is transposed), plus a block
    of the N/2 block in its own launch.  Each image matches the oracle."""
    import torch
    inputs = [synth.deployment(801, n_time=11, n_chan=2),            # 40 rows, transposed
              synth.random_problem(131, 64, 200, 2, 2, 11, fill=0.7),  # 48 rows, transposed
              synth.random_problem(806, 64, 180, 1, 2, 11, fill=0.6),  # 40 rows
              synth.random_problem(805, 64, 150, 2, 2, 11, fill=0.4)]  # the N/2 block
    b, ef, g = _batch(inputs)
    lp = b.launch_plan()
    print(lp, flush=True)
    assert [x[0] for x in lp] == [0, 0, 0, 1] and lp[0][1] == 3
    imgs = b.accumulate(ef, g, b.new_images())
    torch.cuda.synchronize()
    _check_blocks(imgs, inputs)


def test_ungroupable_blocks_run_alone_and_groups_hold_eight():
    """A staged block and a block with autocorrelation removal run through
    their own contexts; nine groupable 32 x 32 blocks form two launches."""
    import torch
    from paper_1904_11422_amd import Batch
    blocks = tuple((32, 40 + 3 * k, 1 + k % 3) for k in range(9)) + ((32, 64, 2), (32, 64, 2))
    inputs = [synth.config4_block(k, n_time=7, blocks=blocks) for k in range(len(blocks))]
    cfgs = [dict(grid_n=i.grid_n, n_chan=i.n_chan, n_pol=i.n_pol, n_ant=i.n_ant) for i in inputs]
    cfgs[9]["staged"] = True
    cfgs[10]["remove_autos"] = True
    b = Batch(cfgs)
    for k, i in enumerate(inputs):
        b.set_antennas(k, i.xy_m, i.freq_hz)
    lp = b.launch_plan()
    print(lp, flush=True)
    assert [x[1] for x in lp[:8]] == [8] * 8 and lp[8][1] == 1
    assert lp[9][1] == 0 and lp[10][1] == 0
    assert len({x[0] for x in lp}) == 4
    ef = [torch.from_numpy(np.ascontiguousarray(i.efield)).cuda() for i in inputs]
    g = [torch.from_numpy(np.ascontiguousarray(i.gains)).cuda() for i in inputs]
    imgs = b.accumulate(ef, g, b.new_images())
    torch.cuda.synchronize()
    _check_blocks(imgs[:10], inputs[:10])
    ref = oracle.image_without_autos_from(inputs[10])
    full = oracle.image_from(inputs[10])
    d = imgs[10].cpu().numpy() - ref
    for c in range(inputs[10].n_chan):
        for pr in range(4):
            assert np.linalg.norm(d[c, pr]) <= 1e-5 * np.linalg.norm(full[c, pr]) + 1e-9


@pytest.mark.parametrize("shape", [(4, 0, 128, 0), (4, 8, 64, 1), (2, 2, 128, 1), (1, 1, 64, 0),
                                   (3, 4, 128, 1), (4, 1, 5, 1)])
def test_every_tuned_shape_matches_oracle(batch_inputs, shape):
    """Each launch shape the tuner can choose -- grid of w_cap * den / 4, team
    size (time chunk), float32 blocks of 128 or 64 samples (and a short one,
    so every part spans several blocks), XCD order on or off -- gives the
    oracle's images."""
    import torch
    den, team, kb, xcd = shape
    b, ef, g = _batch(batch_inputs)
    caps = {lp[0]: grid for lp, (grid, _) in zip(b.launch_plan(), b.plan())}
    for li, cap in caps.items():
        b.set_launch(li, max(1, cap * den // 4), team, kb, xcd)
    assert all(x[2] == team and x[3] == kb and x[4] == xcd for x in b.launch_plan())
    assert all(grid == max(1, caps[lp[0]] * den // 4) for lp, (grid, _) in zip(b.launch_plan(), b.plan()))
    imgs = b.accumulate(ef, g, b.new_images())
    torch.cuda.synchronize()
    _check_blocks(imgs, batch_inputs)
