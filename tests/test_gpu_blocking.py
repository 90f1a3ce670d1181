"""GPU: two time steps per launch (2D keep-all schedule; forward, adjoint or both) against
one step per launch and the FP64 oracle.

Both modes evaluate every cell with the same FP32 instructions, so the recorded data,
the misfit and the imaging operands agree bit for bit.  The per-sample FP64 imaging sum
adds the same exact products in another order (two steps per read-modify-write), so the
FP32 gradient may differ in the last bit of a few cells: relative L2 <= 1e-6.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W
from helpers import f32, oracle_batch_gradient, oracle_forward_sims, rel, split_data, split_model

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12797_amd import fwi
    fwi.lib()
    yield fwi
    fwi.fwi_set_time_blocking(0, 0)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def strip_edge_problem(F, nt, R, ckpt=0):
    """Two samples (one and three supergathers) on grids whose padded sizes are not
    multiples of the 56 x 16 strips.  Sources and receivers sit on the columns and rows
    where strips meet and inside the 4-cell margins the first step also computes,
    including two sources on one cell and sources on several rows of one column."""
    g0 = F.Grid(nz=45, nx=150, dz=10.0, dx=10.0, nb=4, v_ref=3000.0, v_max=3300.0)
    g1 = F.Grid(nz=29, nx=61, dz=8.0, dx=12.0, nb=6, v_ref=3000.0, v_max=3300.0)
    r = np.random.default_rng(31)
    m0 = f32(W.salt_2d(45, 150, seed=4, vtop=1500, vbot=2800, vsalt=3200).ravel())
    m1 = f32(r.uniform(1700, 3200, g1.nphys))

    def cell(g, pz, px):  # from padded coordinates
        return (pz - g.nb) * g.nx + (px - g.nb)

    cols0 = [51, 52, 55, 56, 59, 60, 111, 112, 115, 116]
    rows0 = [12, 15, 16, 19, 20, 31, 32, 35]
    s0 = [([cell(g0, 12, 52), cell(g0, 16, 56), cell(g0, 16, 56), cell(g0, 35, 115), cell(g0, 20, 60)],
           [1.0, -1.0, 1.0, -1.0, 1.0])]
    s1 = [([cell(g1, 15, 52), cell(g1, 16, 52)], [1.0, -1.0]),
          ([cell(g1, 6, 6), cell(g1, 34, 66)], [-1.0, 1.0]),
          ([cell(g1, 19, 59), cell(g1, 20, 56), cell(g1, 31, 12)], [1.0, 1.0, -1.0])]
    rec0 = sorted({cell(g0, z, x) for z in rows0 for x in cols0} | {cell(g0, 5, x) for x in range(4, 154)})
    rec1 = sorted({cell(g1, z, x) for z in (6, 12, 15, 16, 19, 20, 34) for x in (6, 48, 52, 55, 56, 59, 60, 66)})
    rec0 = np.array(rec0, dtype=np.int32)
    rec1 = np.array(rec1, dtype=np.int32)
    wav = W.ricker(20.0, 1e-3, nt)
    batch = F.Batch([g0, g1], [0, 1, 1, 1], s0 + s1, [rec0, rec1, rec1, rec1], wav)
    time = F.time_axis(1e-3, nt, R, ckpt)
    return batch, time, [m0, m1]


def run(F, blocking, batch, time, models, dobs, kappa, is2=2.0):
    F.fwi_set_time_blocking(*blocking)
    nt_rec = time.nt // time.rec_every
    v = dev(np.concatenate([m.ravel() for m in models]))
    dpred = torch.zeros(batch.data_size(nt_rec), device="cuda")
    mis = torch.zeros(batch.nsim, dtype=torch.float64, device="cuda")
    grad = torch.zeros(batch.model_size, device="cuda")
    ws = F.alloc_workspace(batch, time)
    F.fwi_gradient(batch, time, v, dev(dobs), is2, kappa, dpred, mis, grad, None, ws)
    F.fwi_poll_status(ws)
    return dpred.cpu().numpy(), mis.cpu().numpy(), grad.cpu().numpy()


# keep-all (even and odd nt) and checkpointed schedules (odd segments, a short last one):
# with checkpoints the adjoint of every recomputed segment runs in pairs plus an odd step
@pytest.mark.parametrize("nt,R,ckpt", [(160, 2, 0), (161, 1, 0), (99, 3, 0), (100, 2, 7), (99, 3, 10)])
def test_two_steps_equal_one_step(F, nt, R, ckpt):
    say("case two steps per launch vs one, nt=%d rec_every=%d ckpt_every=%d" % (nt, R, ckpt))
    batch, time, models = strip_edge_problem(F, nt, R, ckpt)
    nd = batch.data_size(nt // R)
    dobs = 1e-4 * np.random.default_rng(nt).standard_normal(nd)
    kappa = [1.25, 0.5]
    one = run(F, (1, 1), batch, time, models, dobs, kappa)
    assert np.abs(one[0]).max() > 0 and np.abs(one[2]).max() > 0
    for mode in ((2, 2), (1, 2), (2, 1)):
        two = run(F, mode, batch, time, models, dobs, kappa)
        assert np.array_equal(one[0], two[0]), ("recorded data differ", mode)
        assert np.array_equal(one[1], two[1]), ("misfit differs", mode)
        e = rel(two[2].astype(np.float64), one[2].astype(np.float64))
        same = float(np.mean(one[2] == two[2]))
        say("  steps per launch %s: gradient rel %.2e, %.4f of cells bitwise equal" % (mode, e, same))
        assert e < 1e-6
        if mode[1] == 1:  # same adjoint: same summation order
            assert np.array_equal(one[2], two[2])


def test_two_steps_forward_only(F):
    say("case two steps per launch, forward only")
    batch, _, models = strip_edge_problem(F, 121, 1)
    time = F.time_axis(1e-3, 121, 1, -1)
    v = dev(np.concatenate([m.ravel() for m in models]))
    outs = []
    for blocking in (1, 2):
        F.fwi_set_time_blocking(blocking, 2)
        d = torch.zeros(batch.data_size(121), device="cuda")
        ws = F.alloc_workspace(batch, time)
        F.fwi_forward(batch, time, v, d, ws)
        F.fwi_poll_status(ws)
        outs.append(d.cpu().numpy())
    assert np.abs(outs[0]).max() > 0
    assert np.array_equal(outs[0], outs[1])


def test_two_steps_against_oracle(F):
    say("case two steps per launch vs oracle")
    nt, R = 151, 1
    batch, time, models = strip_edge_problem(F, nt, R)
    r = np.random.default_rng(3)
    truth = [f32(m * (1 + 0.05 * r.standard_normal(m.shape))) for m in models]
    dobs = [f32(d) for d in oracle_forward_sims(batch, 1e-3, nt, R, truth, coef_fp32=False)]
    kappa = [1.25, 0.5]
    is2 = 3.0
    dp, mis, gr = run(F, (2, 2), batch, time, models, np.concatenate([d.ravel() for d in dobs]), kappa, is2)
    odp, omis, ogr = oracle_batch_gradient(batch, 1e-3, nt, R, [m.ravel() for m in models], dobs, is2, kappa)
    gdp = split_data(dp.astype(np.float64), batch, nt // R)
    for s in range(batch.nsim):
        e = rel(gdp[s], odp[s])
        say("  sim %d data rel %.2e misfit rel %.2e" % (s, e, abs(mis[s] / omis[s] - 1)))
        assert e < TOL and abs(mis[s] / omis[s] - 1) < TOL
    gg = split_model(gr.astype(np.float64), batch)
    for k in range(batch.nsample):
        e = rel(gg[k], ogr[k])
        say("  sample %d gradient rel %.2e" % (k, e))
        assert e < TOL


def test_two_strips_per_workgroup_odd_strip_count(F):
    # one sample of 10 supergathers on a grid of 3 strips (52 x 42 padded): the two-step
    # adjoint runs 8 waves per workgroup as two strips of 4 waves each (10 sims split
    # 3+3+2+2 per strip, instead of 2+2+1+1+1+1+1+1 on one strip of 8 waves), and the last
    # workgroup's second strip does not exist (its waves only join the barriers)
    say("case two strips per workgroup, odd strip count")
    g = F.Grid(nz=30, nx=40, dz=10.0, dx=10.0, nb=6, v_ref=3000.0, v_max=3300.0)
    r = np.random.default_rng(5)
    model = f32(r.uniform(1800, 3200, g.nphys))
    rec = (np.arange(0, 40, 2) + 40).astype(np.int32)
    srcs = [(r.integers(0, g.nphys, 2).astype(np.int32), r.choice([-1.0, 1.0], 2)) for _ in range(10)]
    nt, R = 120, 2
    batch = F.Batch([g], [0] * 10, srcs, [rec] * 10, W.ricker(15.0, 1e-3, nt))
    time = F.time_axis(1e-3, nt, R, 0)
    nd = batch.data_size(nt // R)
    dobs = f32(1e-4 * np.random.default_rng(9).standard_normal(nd))
    one = run(F, (1, 1), batch, time, [model], dobs, [0.75])
    two = run(F, (1, 2), batch, time, [model], dobs, [0.75])
    assert np.abs(one[2]).max() > 0
    assert np.array_equal(one[0], two[0]) and np.array_equal(one[1], two[1])
    e = rel(two[2].astype(np.float64), one[2].astype(np.float64))
    say("  gradient rel %.2e" % e)
    assert e < 1e-6
    # and against the oracle
    dp, mis, gr = two
    truth_d = split_data(dobs, batch, nt // R)
    odp, omis, ogr = oracle_batch_gradient(batch, 1e-3, nt, R, [model.ravel()], truth_d, 2.0, [0.75])
    assert rel(gr.astype(np.float64), ogr[0]) < TOL
