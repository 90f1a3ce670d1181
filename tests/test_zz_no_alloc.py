"""The allocation-free gradient (fwi_gradient_noalloc) against fwi_gradient on a caller
workspace: two calls in a row through the C ABI, the second on a smaller batch, must
give the same data, misfits, gradients and norms bit for bit (same kernels, same
tables); a batch whose workspace exceeds the library's array is refused before anything
is enqueued."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W
from helpers import f32

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12797_amd import fwi
    fwi.lib()
    return fwi


def _problem(F, nz, nx, nsample, s, G, nshot, nt, ckpt, seed):
    from paper_2512_12797_amd import problems
    cfg = W.C1
    grid = F.Grid(nz=nz, nx=nx, dz=10.0, dx=10.0, nb=10, v_ref=4000.0, v_max=4400.0)
    wav = W.ricker(15.0, 1e-3, nt)
    batch, groups = problems.encoded_batch(cfg, [grid] * nsample, wav, seed=seed, step=0, s=s, G=G,
                                           nshot_of=lambda g: nshot)
    time = F.time_axis(1e-3, nt, 1, ckpt)
    v = torch.tensor(np.tile(f32(W.linear_gradient(nz, nx)).ravel(), nsample), dtype=torch.float32, device="cuda")
    r = np.random.default_rng(seed)
    dobs = torch.tensor(r.standard_normal(batch.data_size(nt)) * 1e-3, dtype=torch.float32, device="cuda")
    kappa = [g[2] for g in groups]
    return batch, time, v, dobs, kappa


def _outputs(F, batch, time):
    nd = batch.data_size(time.nt // time.rec_every)
    return (torch.full((nd,), 7.0, device="cuda"), torch.full((batch.nsim,), 7.0, dtype=torch.float64, device="cuda"),
            torch.full((batch.model_size,), 7.0, device="cuda"), torch.full((batch.nsample,), 7.0, device="cuda"))


def test_noalloc_matches_workspace_gradient(F):
    cases = [("2 samples x 2 supergathers, 64x96, 400 steps, K 10", (64, 96, 2, 4, 2, 8, 400, 10, 3)),
             ("1 sample x 1 supergather, 30x45, 150 steps, keep-all", (30, 45, 1, 2, 1, 2, 150, 0, 4))]
    for name, args in cases:
        say("case noalloc vs workspace: %s" % name)
        batch, time, v, dobs, kappa = _problem(F, *args)
        assert F.fwi_workspace_size(batch, time) <= F.NOALLOC_MAX_BYTES
        ref = _outputs(F, batch, time)
        ws = F.alloc_workspace(batch, time)
        F.fwi_gradient(batch, time, v, dobs, 3.0, kappa, ref[0], ref[1], ref[2], ref[3], ws)
        F.fwi_poll_status(ws)
        got = _outputs(F, batch, time)
        F.fwi_gradient_noalloc(batch, time, v, dobs, 3.0, kappa, got[0], got[1], got[2], got[3])
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
        assert float(got[2].abs().max()) > 0
        del ws


def test_noalloc_refuses_oversized_batch(F):
    say("case noalloc oversized batch")
    batch, time, v, dobs, kappa = _problem(F, 300, 400, 2, 4, 2, 8, 600, 0, 5)
    assert F.fwi_workspace_size(batch, time) > F.NOALLOC_MAX_BYTES
    got = _outputs(F, batch, time)
    with pytest.raises(F.FwiError) as e:
        F.fwi_gradient_noalloc(batch, time, v, dobs, 1.0, kappa, got[0], got[1], got[2], got[3])
    assert e.value.status == F.FWI_E_WORKSPACE
    torch.cuda.synchronize()
    assert bool((got[2] == 7.0).all()) and bool((got[1] == 7.0).all())
