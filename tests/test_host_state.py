"""Host: the chain state file round-trips exactly and holds only plain arrays."""
import numpy as np


def test_state_roundtrip(tmp_path):
    from paper_2512_12797_amd import chains
    r = np.random.default_rng(0)
    v = r.normal(3000.0, 100.0, (3, 17)).astype(np.float32)
    path = str(tmp_path / "s.npz")
    chains.save_state(path, v, 41, 12345)
    with np.load(path, allow_pickle=False) as z:  # loads without unpickling
        assert sorted(z.files) == ["seed", "step", "v"]
    v2, step, seed = chains.load_state(path, device="cpu")
    assert step == 41 and seed == 12345 and np.array_equal(v2.numpy(), v)
