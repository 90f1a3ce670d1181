"""GPU: the SVGD step (include/fwi_svgd.h) against the FP64 oracle (oracle/svgd.py),
through the C ABI.  The library computes distances, bandwidth, kernel and direction in
FP64 and rounds once, so the direction matches the oracle to FP32 rounding of its
largest value and the bandwidth to FP64 rounding of the distance sums."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import svgd as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12797_amd import svgd
    return svgd


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def particles(n, N, seed, spread=20.0):
    r = np.random.default_rng(seed)
    base = 3000.0 + 800.0 * r.random(N)
    x = f32(base[None, :] + spread * r.normal(size=(n, N)))
    g = f32(1e-3 * r.normal(size=(n, N)) + 2e-4 * (x - base[None, :]))
    return x, g


def run(M, x, g, eps, h=0.0, lo=1000.0, hi=8000.0):
    n, N = x.shape
    xt, gt = dev(x), dev(g)
    out = torch.empty_like(xt)
    phi = torch.empty_like(xt)
    hh = torch.empty(1, dtype=torch.float64, device="cuda")
    work = torch.empty((M.fwi_svgd_work_size(n, N) + 7) // 8, dtype=torch.float64, device="cuda")
    M.fwi_svgd_step(n, N, xt, gt, eps, h, lo, hi, out, phi, hh, work)
    return out.cpu().numpy().astype(np.float64), phi.cpu().numpy().astype(np.float64), float(hh.item())


# sizes: one chunk, a ragged tail, several distance chunks, the 2D workload's particles
# (16 x 60000) and the largest particle count
@pytest.mark.parametrize("n,N", [(1, 7), (2, 1000), (5, 5003), (16, 60000), (16, 70001), (64, 9001)])
def test_step_matches_oracle(M, n, N):
    say("case svgd step n=%d N=%d" % (n, N))
    x, g = particles(n, N, seed=n * 1000 + N % 997)
    eps = 50.0
    got_x, got_phi, got_h = run(M, x, g, eps)
    phi, K, h = S.direction(x, g)
    ref_x = np.clip(x + eps * phi, 1000.0, 8000.0)
    e_phi = np.abs(got_phi - phi).max() / np.abs(phi).max()
    say("  h %.6e vs %.6e, phi rel error %.2e, x max abs error %.2e" % (got_h, h, e_phi, np.abs(got_x - ref_x).max()))
    assert abs(got_h / h - 1) < 1e-12
    assert e_phi < 1e-6
    assert np.abs(got_x - ref_x).max() < 1e-3  # FP32 spacing at 4000 m/s is 2.4e-4


def test_fixed_bandwidth_and_clamp(M):
    say("case svgd fixed bandwidth")
    x, g = particles(6, 4099, seed=5)
    h = 1.0e6
    got_x, got_phi, got_h = run(M, x, g, 3000.0, h=h, lo=3100.0, hi=3700.0)
    phi, _, _ = S.direction(x, g, h)
    assert got_h == h
    assert np.abs(got_phi - phi).max() / np.abs(phi).max() < 1e-6
    ref = np.clip(x + 3000.0 * phi, 3100.0, 3700.0)
    assert np.any(ref == 3100.0) and np.any(ref == 3700.0)
    assert np.abs(got_x - ref).max() < 1e-3


def test_coincident_particles_and_zero_step(M):
    say("case svgd coincident particles")
    r = np.random.default_rng(7)
    x = np.tile(f32(3000.0 + r.random(777) * 500.0), (4, 1))
    g = f32(r.normal(size=(4, 777)))
    got_x, got_phi, got_h = run(M, x, g, 0.0, lo=3100.0, hi=3400.0)
    phi, _, h = S.direction(x, g)
    assert got_h == 1.0 == h
    assert np.abs(got_phi - phi).max() <= 1e-7 * np.abs(phi).max()
    assert np.array_equal(got_x, f32(np.clip(x, 3100.0, 3400.0)))  # eps = 0: only the clamp


def test_repeatable(M):
    x, g = particles(16, 60000, seed=9)
    a = run(M, x, g, 10.0)
    b = run(M, x, g, 10.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
