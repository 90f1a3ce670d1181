"""GPU edge cases through the C ABI.

* Degenerate grids and time axes against the FP64 oracle: one-cell-wide grids, no sponge,
  a number of steps that is not a multiple of the checkpoint interval, an interval at
  least as long as the run, a single step; every batch also holds a supergather with no
  sources and no receivers (empty input: zero data, no contribution to the gradient).
* A zero residual gives an exactly zero gradient.
* Grids at the library's size limit (2D and 3D): with the source near the far corner
  (the highest addresses of every field), the data and the gradient near the source equal
  those of a small grid with the same neighbourhood bit for bit -- every cell update is
  the same arithmetic, so only addressing could make them differ.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import workloads as W
from helpers import f32, ogrid, rel, split_data, split_model

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
    return fwi


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


# (nz, nx, nb, nt, rec_every, ckpt_every)
CASES = [
    (1, 3, 0, 20, 1, 0),
    (5, 1, 2, 24, 2, 5),
    (9, 70, 0, 30, 3, 7),
    (12, 40, 3, 12, 4, 20),
    (12, 40, 3, 1, 1, 0),
]


@pytest.mark.parametrize("nz,nx,nb,nt,R,K", CASES)
def test_degenerate_grids_and_time_axes(F, nz, nx, nb, nt, R, K):
    say("case degenerate nz=%d nx=%d nb=%d nt=%d R=%d K=%d" % (nz, nx, nb, nt, R, K))
    g = F.Grid(nz=nz, nx=nx, dz=10.0, dx=10.0, nb=nb, v_ref=3000.0, v_max=3000.0)
    r = np.random.default_rng(nz * 100 + nx + nt)
    n = nz * nx
    m = f32(r.uniform(1800, 3000, n))
    srcs = [(r.choice(n, 2, replace=False).astype(np.int32), [1.0, -1.0]), (np.zeros(0, dtype=np.int32), [])]
    # a receiver on a source cell: even a single step records something
    rec = np.unique(np.r_[r.integers(0, n, min(n, 5)), srcs[0][0][:1]]).astype(np.int32)
    recs = [rec, np.zeros(0, dtype=np.int32)]
    wav = W.ricker(4.5 / (nt * 1e-3), 1e-3, nt)  # centred a third of the way into the run
    batch = F.Batch([g], [0, 0], srcs, recs, wav)
    time = F.time_axis(1e-3, nt, R, K)
    nt_rec = nt // R
    v = dev(m)
    ws = F.alloc_workspace(batch, time)
    d = torch.zeros(batch.data_size(nt_rec), device="cuda")
    F.fwi_forward(batch, time, v, d, ws)
    rho = [f32(r.standard_normal((nt_rec, len(rec))) * 1e-2), np.zeros((nt_rec, 0))]
    grad = torch.zeros(batch.model_size, device="cuda")
    F.fwi_adjoint(batch, time, v, dev(np.concatenate([x.ravel() for x in rho])), [1.7], grad, None, ws)
    F.fwi_poll_status(ws)
    dd = split_data(d.cpu().numpy().astype(np.float64), batch, nt_rec)
    od = oracle.forward(ogrid(g), m, 1e-3, nt, R, srcs[0][0], f32(srcs[0][1]), f32(wav), rec)
    e = rel(dd[0], od) if np.linalg.norm(od) > 0 else float(np.abs(dd[0]).max())
    og, _ = oracle.adjoint(ogrid(g), m, 1e-3, nt, R, srcs[0][0], f32(srcs[0][1]), f32(wav), rec, rho[0])
    og2, _ = oracle.adjoint(ogrid(g), m, 1e-3, nt, R, [], [], f32(wav), [], rho[1])
    gg = grad.cpu().numpy().astype(np.float64)
    ref = 1.7 * (og + og2)
    eg = rel(gg, ref) if np.linalg.norm(ref) > 0 else float(np.abs(gg).max())
    say("  data rel %.2e, gradient rel %.2e (|data| %.2e, |gradient| %.2e)" % (e, eg, np.abs(od).max(),
                                                                             np.abs(ref).max()))
    assert np.abs(od).max() > 0 and np.abs(ref).max() > 0
    assert e < TOL and eg < TOL
    assert dd[1].size == 0


def test_zero_residual_gives_zero_gradient(F):
    say("case zero residual")
    g = F.Grid(nz=30, nx=50, dz=10.0, dx=10.0, nb=5, v_ref=3000.0, v_max=3000.0)
    m = np.random.default_rng(3).uniform(1800, 3000, g.nphys)
    rec = (np.arange(50) + 50).astype(np.int32)
    batch = F.Batch([g], [0, 0], [([55], [1.0]), ([70, 90], [1.0, -1.0])], [rec, rec], W.ricker(15.0, 1e-3, 150))
    time = F.time_axis(1e-3, 150, 1, 0)
    v = dev(m)
    ws = F.alloc_workspace(batch, time)
    d = torch.zeros(batch.data_size(150), device="cuda")
    F.fwi_forward(batch, time, v, d, ws)
    mis = torch.zeros(2, dtype=torch.float64, device="cuda")
    grad = torch.ones(batch.model_size, device="cuda")
    F.fwi_gradient(batch, time, v, d.clone(), 1.0, None, None, mis, grad, None, ws)
    F.fwi_poll_status(ws)
    assert float(mis.abs().max()) == 0.0
    assert float(grad.abs().max()) == 0.0


def _corner_problem(F, ndim, big):
    """One simulation with its source 21..41 cells before the far corner of a grid at the
    size limit (big) or of a small grid with the same neighbourhood; receivers around the
    source; returns (batch, time, model, receiver offsets, crop of the gradient)."""
    if ndim == 2:
        n, far, nb, nt = (16000 if big else 100), 41, 20, 12
        g = F.Grid(nz=n, nx=n, dz=10.0, dx=10.0, nb=nb, v_ref=3000.0, v_max=3000.0)
        sz = sx = n - far
        offs = [(dz, dx) for dz in range(-6, 7, 3) for dx in range(-6, 7, 2)]
        rec = np.array([(sz + a) * n + sx + b for a, b in offs], dtype=np.int32)
        src = [sz * n + sx]
        m = np.full(g.nphys, 2500.0, dtype=np.float32)
        box = lambda a: a.reshape(n, n)[n - 2 * far:, n - 2 * far:]  # noqa: E731
    else:
        n, far, nb, nt = (560 if big else 60), 21, 10, 8
        g = F.Grid(nz=n, ny=n, nx=n, dz=20.0, dy=20.0, dx=20.0, nb=nb, v_ref=3000.0, v_max=3000.0, ndim=3)
        c = n - far
        offs = [(a, b, e) for a in (-4, 0, 4) for b in (-4, 0, 4) for e in (-6, -2, 2, 6)]
        rec = np.array([((c + a) * n + c + b) * n + c + e for a, b, e in offs], dtype=np.int32)
        src = [(c * n + c) * n + c]
        m = np.full(g.nphys, 2500.0, dtype=np.float32)
        box = lambda a: a.reshape(n, n, n)[n - 2 * far:, n - 2 * far:, n - 2 * far:]  # noqa: E731
    dt = 2e-3 if ndim == 3 else 1e-3
    batch = F.Batch([g], [0], [(src, [1.0])], [rec], W.ricker(15.0, dt, nt))
    return batch, F.time_axis(dt, nt, 1, 0), m, box


@pytest.mark.parametrize("ndim", [2, 3])
def test_grid_at_size_limit_matches_small_grid(F, ndim):
    say("case size limit %dD" % ndim)
    outs = []
    for big in (False, True):
        batch, time, m, box = _corner_problem(F, ndim, big)
        g = batch.grids[0]
        F.fwi_check(batch, time)
        v = dev(m)
        ws = F.alloc_workspace(batch, time)
        say("  %s grid: %d physical cells, workspace %.1f GB" % ("limit" if big else "small", g.nphys, ws.numel() / 1e9))
        d = torch.zeros(batch.data_size(time.nt), device="cuda")
        F.fwi_forward(batch, time, v, d, ws)
        rho = dev(np.random.default_rng(5).standard_normal(batch.data_size(time.nt)) * 1e-2)
        grad = torch.zeros(batch.model_size, device="cuda")
        F.fwi_adjoint(batch, time, v, rho, None, grad, None, ws)
        F.fwi_poll_status(ws)
        outs.append((d.cpu().numpy(), box(grad.cpu().numpy()).copy()))
        del ws, v, grad, d
        torch.cuda.empty_cache()
    assert np.abs(outs[0][0]).max() > 0 and np.abs(outs[0][1]).max() > 0
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    # the small grid itself against the oracle
    batch, time, m, box = _corner_problem(F, ndim, False)
    od = oracle.forward(ogrid(batch.grids[0]), m.astype(np.float64), time.dt, time.nt, 1, batch.src_cell, [1.0],
                        f32(batch.wavelet), batch.rec_cell)
    assert rel(outs[0][0].reshape(od.shape), od) < TOL
