"""C ABI checks that need no GPU: symbols, host validation, workspace sizing, encoding draw."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    from paper_2512_12797_amd import fwi
    if not os.path.exists(fwi.LIB_PATH):
        pytest.skip("library not built")
    fwi.lib()
    return fwi


def declared_symbols():
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(fwi_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_every_declared_symbol_is_exported(F):
    names = declared_symbols()
    assert len(names) >= 30 and "fwi_nn_conv3x3" in names and "fwi_gradient" in names
    L = C.CDLL(F.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def small(F, **kw):
    g = F.Grid(nz=20, nx=30, dz=10.0, dx=10.0, nb=4, v_ref=3000.0, v_max=3000.0)
    for k, v in kw.items():
        setattr(g, k, v)
    rec = np.arange(30, dtype=np.int32) + 30
    wav = W.ricker(10.0, 1e-3, 100)
    return g, rec, wav


def expect(F, status, fn, *a):
    with pytest.raises(F.FwiError) as e:
        fn(*a)
    assert e.value.status == status, str(e.value)


def test_validation_errors(F):
    g, rec, wav = small(F)
    b = F.Batch([g], [0], [([31], [1.0])], [rec], wav)
    t = F.time_axis(1e-3, 100, 2, 0)
    assert 0 < F.fwi_check(b, t) < 0.79
    # stability limit: v_max dt sqrt(2)/h must stay below sqrt(315/512)
    lim = np.sqrt(315 / 512) / np.sqrt(2) * 10.0 / 3000.0
    expect(F, F.FWI_E_CFL, F.fwi_check, b, F.time_axis(lim * 1.01, 100, 1, 0))
    F.fwi_check(b, F.time_axis(lim * 0.99, 100, 1, 0))
    expect(F, F.FWI_E_ARG, F.fwi_check, b, F.time_axis(1e-3, 101, 2, 0))
    expect(F, F.FWI_E_ARG, F.fwi_check, b, F.time_axis(1e-3, 100, 1, -2))
    gbad, _, _ = small(F, ny=2)
    expect(F, F.FWI_E_ARG, F.fwi_check, F.Batch([gbad], [0], [([31], [1.0])], [rec], wav), t)
    expect(F, F.FWI_E_ARG, F.fwi_check, F.Batch([g], [0], [([600], [1.0])], [rec], wav), t)
    expect(F, F.FWI_E_ARG, F.fwi_check, F.Batch([g], [0], [([31], [1.0])], [np.r_[rec, rec[:1]]], wav), t)
    expect(F, F.FWI_E_ARG, F.fwi_check, F.Batch([g, g], [1, 0], [([31], [1.0])] * 2, [rec] * 2, wav), t)
    expect(F, F.FWI_E_ARG, F.fwi_check, F.Batch([g, g], [0, 0], [([31], [1.0])] * 2, [rec] * 2, wav), t)
    expect(F, F.FWI_E_ARG, F.fwi_check, F.Batch([g], [0], [([31], [np.nan])], [rec], wav), t)
    # empty batch
    expect(F, F.FWI_E_ARG, F.fwi_check, F.Batch([g], [], [], [], wav), t)
    # size limits: more than 2^28 padded cells; fewer, but offsets 80 rows past the grid
    # beyond 2^30 bytes (a very wide, shallow grid)
    big = F.Grid(nz=16400, nx=16400, dz=10.0, dx=10.0, nb=20, v_ref=3000.0, v_max=3000.0)
    expect(F, F.FWI_E_UNSUPPORTED, F.fwi_check, F.Batch([big], [0], [([5], [1.0])], [rec[:1]], wav), t)
    wide = F.Grid(nz=23, nx=(1 << 22) - 40, dz=10.0, dx=10.0, nb=20, v_ref=3000.0, v_max=3000.0)
    expect(F, F.FWI_E_UNSUPPORTED, F.fwi_check, F.Batch([wide], [0], [([5], [1.0])], [rec[:1]], wav), t)
    ok = F.Grid(nz=16000, nx=16000, dz=10.0, dx=10.0, nb=20, v_ref=3000.0, v_max=3000.0)
    F.fwi_check(F.Batch([ok], [0], [([5], [1.0])], [rec[:1]], wav), t)
    g3 = F.Grid(nz=4, ny=4, nx=4, dz=10, dy=10, dx=10, nb=1, v_ref=2000, v_max=2000, ndim=3)
    expect(F, F.FWI_E_UNSUPPORTED, F.fwi_check, F.Batch([g, g3], [0, 1], [([31], [1.0]), ([1], [1.0])],
                                                        [rec, np.array([2], dtype=np.int32)], wav), t)


def test_workspace_sizes(F):
    g, rec, wav = small(F)
    b = F.Batch([g], [0, 0], [([31], [1.0]), ([40], [-1.0])], [rec, rec], wav)
    cells = 2 * (28 * 38)
    full = F.fwi_workspace_size(b, F.time_axis(1e-3, 100, 2, 0))
    ck = F.fwi_workspace_size(b, F.time_axis(1e-3, 100, 2, 10))
    assert full >= 100 * cells * 4
    assert ck < full
    assert ck >= (10 + 2 * 9) * cells * 4


def test_kept_tail_validation_and_sizes(F):
    """keep_tail: range and schedule checks; the workspace holds the recomputation ring,
    the kept tail and the checkpoints of the first nt - keep_tail steps, the ring inside the
    tail's levels when the tail is at least as long (the adjoint reads the tail first)."""
    g, rec, wav = small(F)
    b = F.Batch([g], [0, 0], [([31], [1.0]), ([40], [-1.0])], [rec, rec], wav)
    for K, T in ((10, -1), (10, 101), (0, 5), (-1, 5)):
        expect(F, F.FWI_E_ARG, F.fwi_check, b, F.time_axis(1e-3, 100, 2, K, T))
    lev = 2 * (28 * 38) * 4  # one level of both sims (bytes)
    size = lambda K, T: F.fwi_workspace_size(b, F.time_axis(1e-3, 100, 2, K, T))
    base = size(10, 0)  # ring 10 + 2 x 9 checkpoint levels = 28
    # tail 30: head 70 -> 7 segments: tail 30 (holding the ring) + 2 x 6 checkpoint levels = 42
    assert abs(size(10, 30) - base - 14 * lev) <= 512
    # tail 6, shorter than the ring: head 94 -> 10 segments: ring 10 + tail 6 + 2 x 9 = 34
    assert abs(size(10, 6) - base - 6 * lev) <= 512
    # tail 95: head 5 -> a ring of 5 levels inside the tail, one segment, no checkpoint: 95
    assert abs(size(10, 95) - base - 67 * lev) <= 512
    # every step kept through the tail: no ring, no checkpoint: 100
    assert abs(size(10, 100) - base - 72 * lev) <= 512
    assert size(10, 100) > F.fwi_workspace_size(b, F.time_axis(1e-3, 100, 2, 0))  # two more field levels


def test_schedule_for_a_budget(F):
    g, rec, wav = small(F)
    b = F.Batch([g], [0, 0], [([31], [1.0]), ([40], [-1.0])], [rec, rec], wav)
    t = F.time_axis(1e-3, 100, 2)
    full = F.fwi_workspace_size(b, t)
    s = F.fwi_schedule(b, t, full)
    assert (s.ckpt_every, s.keep_tail) == (0, 0) and (s.dt, s.nt, s.rec_every) == (t.dt, 100, 2)
    lev = 2 * (28 * 38) * 4
    for budget in (full - 1, full - 30 * lev, full - 60 * lev):
        s = F.fwi_schedule(b, t, budget)
        K, T = s.ckpt_every, s.keep_tail
        assert K >= 1 and 0 <= T < 100
        assert F.fwi_workspace_size(b, s) <= budget
        # no schedule keeps a longer tail within the budget (fewer forward steps)
        for K2 in range(1, 101 - (T + 1)):
            assert F.fwi_workspace_size(b, F.time_axis(1e-3, 100, 2, K2, T + 1)) > budget
    small_budget = F.fwi_workspace_size(b, F.time_axis(1e-3, 100, 2, 10, 0)) - 30 * lev
    expect(F, F.FWI_E_WORKSPACE, F.fwi_schedule, b, t, small_budget)
    # with the recomputation beside the adjoint the ring is doubled: the pick still fits
    F.fwi_set_overlap(True)
    try:
        for budget in (full - 1, full - 30 * lev):
            s = F.fwi_schedule(b, t, budget)
            assert s.ckpt_every >= 1 and F.fwi_workspace_size(b, s) <= budget
            for K2 in range(1, 100 - s.keep_tail):
                assert F.fwi_workspace_size(b, F.time_axis(1e-3, 100, 2, K2, s.keep_tail + 1)) > budget
    finally:
        F.fwi_set_overlap(False)


def test_null_workspace_rejected_before_any_device_work(F):
    g, rec, wav = small(F)
    b = F.Batch([g], [0], [([31], [1.0])], [rec], wav)
    t = F.time_axis(1e-3, 100, 2, 0)
    L = F.lib()
    st = L.fwi_forward(b.c, C.byref(t), C.c_void_p(1 << 20), None, None, 0, None)
    assert st == F.FWI_E_WORKSPACE
    st = L.fwi_gradient(b.c, C.byref(t), C.c_void_p(1 << 20), C.c_void_p(1 << 20), C.c_float(-1.0), None, None,
                        None, C.c_void_p(1 << 20), None, C.c_void_p(1 << 21), 1 << 40, None)
    assert st == F.FWI_E_ARG  # inv_sigma2 <= 0
    assert b"inv_sigma2" in L.fwi_last_error()


@pytest.mark.parametrize("nshot,s,G", [(80, 8, 10), (80, 16, 10), (8, 1, 8), (50, 8, 1), (7, 3, 5)])
def test_draw_encoding_bit_exact_vs_oracle(F, nshot, s, G):
    for step in (0, 1, 99):
        for sample in (0, 5):
            a = F.fwi_draw_encoding(2024, step, sample, nshot, s, G)
            b = oracle.draw_encoding(2024, step, sample, nshot, s, G)
            assert np.array_equal(a[0], b[0])
            assert np.array_equal(a[1].astype(np.float64), b[1])
            assert a[2] == b[2]


def test_langevin_argument_checks(F):
    L = F.lib()
    off = np.array([0, 10], dtype=np.int64)
    p = C.c_void_p(1 << 20)
    st = L.fwi_langevin(1, off.ctypes.data_as(C.POINTER(C.c_int64)), p, p, None, 0, 0, C.c_float(-1.0),
                        C.c_float(1.0), C.c_float(0.0), C.c_float(1.0), None)
    assert st == F.FWI_E_ARG
    st = L.fwi_langevin(1, off.ctypes.data_as(C.POINTER(C.c_int64)), p, p, None, 0, 0, C.c_float(1.0),
                        C.c_float(1.0), C.c_float(2.0), C.c_float(1.0), None)
    assert st == F.FWI_E_ARG
    assert F.lib().fwi_status_string(F.FWI_E_CFL)


def test_3d_tile_shape_defaults(F):
    """Default 3D tiles: 32 cells wide where that runs fewer lanes than 64 (the bench grid's
    220-cell rows: 7 x 32 against 4 x 64), else 64; the height with the fewest planes read
    per tile column (120 padded planes: three 40-plane tiles)."""
    from paper_2512_12797_amd import problems
    cfg = W.C5
    grid = problems.grid_of(cfg)
    wav = W.ricker(cfg.freq, cfg.dt, 20)
    b, _ = problems.encoded_batch(cfg, [grid] * cfg.nsample, wav, 0, 0)
    assert F.fwi_tile_shape(b, F.time_axis(cfg.dt, 20, 1, 10)) == (40, 32)
    # 128 x 24 rows (no sponge): 64-wide tiles run 128 x 24 lanes, 32-wide 128 x 32
    g = F.Grid(nz=20, ny=24, nx=128, dz=10, dy=10, dx=10, nb=0, v_ref=2000, v_max=2000, ndim=3)
    b2 = F.Batch([g] * 64, list(range(64)), [([5], [1.0])] * 64, [np.array([7], dtype=np.int32)] * 64,
                 W.ricker(10.0, 1e-3, 20))
    assert F.fwi_tile_shape(b2, F.time_axis(1e-3, 20, 1, 0))[1] == 64


def test_time_blocking_values(F):
    # 0 (automatic), 1 or 2 time steps per launch for each sweep; anything else is rejected
    # on the host
    for bad in ((3, 0), (0, 3), (-1, 1), (1, -1)):
        expect(F, F.FWI_E_ARG, F.fwi_set_time_blocking, *bad)
    for ok in ((1, 1), (2, 2), (1, 2), (2, 1), (0, 0)):
        F.fwi_set_time_blocking(*ok)


def test_workspace_independent_of_time_blocking(F):
    # 2D always reserves four field levels and the two-step strip tables, so a workspace
    # sized under one setting serves every other
    g, rec, wav = small(F)
    b = F.Batch([g], [0], [([31], [1.0])], [rec], wav)
    t = F.time_axis(1e-3, 100, 2, 0)
    sizes = set()
    try:
        for mode in ((1, 1), (2, 2), (1, 2), (0, 0)):
            F.fwi_set_time_blocking(*mode)
            sizes.add(F.fwi_workspace_size(b, t))
    finally:
        F.fwi_set_time_blocking(0, 0)
    assert len(sizes) == 1


def test_daps_argument_checks(F):
    # host-side checks of the diffusion outer loop's entry points: nothing is enqueued
    from paper_2512_12797_amd import daps
    L = daps._lib()
    p = C.c_void_p(16)  # never dereferenced: every call below fails its checks first
    assert L.fwi_daps_mix(0, 10, p, None, p, p, p, 1500.0, 5000.0, 1, 0, p, None) == F.FWI_E_ARG
    assert L.fwi_daps_mix(2, 10, None, None, p, p, p, 1500.0, 5000.0, 1, 0, p, None) == F.FWI_E_ARG
    assert L.fwi_daps_mix(2, 10, p, None, p, p, p, 5000.0, 1500.0, 1, 0, p, None) == F.FWI_E_ARG
    assert L.fwi_daps_mix(70000, 10, p, None, p, p, p, 1500.0, 5000.0, 1, 0, p, None) == F.FWI_E_ARG
    assert L.fwi_daps_prep(2, 10, 8, 9, p, p, C.c_void_p(18), None, None) == F.FWI_E_ARG  # misaligned
    assert L.fwi_daps_prep(2, 10, 8, 9, p, p, p, None, None) == F.FWI_E_ARG  # hp < h
    assert L.fwi_daps_model(2, 10, 8, 10, 0, p, 1500.0, 5000.0, p, None) == F.FWI_E_ARG
    assert b"model" in L.fwi_daps_last_error()


def test_svgd_argument_checks(F):
    # host-side checks of the SVGD step: nothing is enqueued
    from paper_2512_12797_amd import svgd
    L = svgd._lib()
    assert svgd.fwi_svgd_work_size(0, 10) == 0 and svgd.fwi_svgd_work_size(65, 10) == 0
    assert svgd.fwi_svgd_work_size(16, 60000) == 8 * (120 * 15 + 256 + 2)
    assert svgd.fwi_svgd_work_size(1, 5) == 8 * (1 + 2)
    a, b, c = C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20)  # never dereferenced
    w, nb = C.c_void_p(4 << 20), 1 << 20
    ok = (4, 100, a, b, 0.1, 0.0, 1500.0, 5000.0, c, None, None, w, nb, None)

    def call(**kw):
        args = list(ok)
        for k, v in kw.items():
            args[{"n": 0, "N": 1, "x": 2, "g": 3, "eps": 4, "lo": 6, "hi": 7, "out": 8, "phi": 9, "w": 11,
                  "nb": 12}[k]] = v
        return L.fwi_svgd_step(*args)

    assert call(n=0) == F.FWI_E_ARG and call(n=65) == F.FWI_E_ARG and call(N=0) == F.FWI_E_ARG
    assert call(x=None) == F.FWI_E_ARG and call(out=None) == F.FWI_E_ARG
    assert call(eps=-1.0) == F.FWI_E_ARG and call(eps=float("inf")) == F.FWI_E_ARG
    assert call(lo=5000.0, hi=1500.0) == F.FWI_E_ARG
    assert call(out=C.c_void_p((1 << 20) + 400)) == F.FWI_E_ARG  # x_out overlaps x (4 x 100 floats)
    assert call(phi=a) == F.FWI_E_ARG and call(phi=b) == F.FWI_E_ARG and call(phi=c) == F.FWI_E_ARG
    assert call(w=None) == F.FWI_E_WORKSPACE and call(w=C.c_void_p((4 << 20) + 4)) == F.FWI_E_WORKSPACE
    assert call(nb=8) == F.FWI_E_WORKSPACE
    assert b"work" in L.fwi_svgd_last_error()
