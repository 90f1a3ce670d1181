"""GPU: a Langevin chain saved after some steps and resumed from the saved state continues
bit for bit like the uninterrupted chain (the encodings and the noise are counter-based:
seed, step, sample), on the 2D encoded workload's survey."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_chain_resume_is_bitwise(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12797_amd import chains
    say("case chain resume (2D workload, 4 samples, 2 + 2 encoded Langevin steps)")
    sv = chains.Survey(seed=1000, log=lambda *a: None)
    eta, seed, ns = 1e-4, 7, 4
    _, _, _, v_full = chains.run_chain(sv, "encoded", 4, eta, seed, nsample=ns, keep_samples=True)
    _, _, _, v_half = chains.run_chain(sv, "encoded", 2, eta, seed, nsample=ns, keep_samples=True)
    path = str(tmp_path / "chain.npz")
    chains.save_state(path, v_half, 2, seed)
    v0, step0, seed0 = chains.load_state(path)
    assert step0 == 2 and seed0 == seed and torch.equal(v0, v_half)
    log = str(tmp_path / "chain.jsonl")
    _, _, _, v_res = chains.run_chain(sv, "encoded", 2, eta, seed0, nsample=ns, keep_samples=True, v0=v0,
                                      step0=step0, log_jsonl=log, elapsed0=5.0)
    import json
    recs = [json.loads(l) for l in open(log)]
    assert [r["step"] for r in recs] == [2, 3]
    # seconds since the chain's start: the resumed run continues from the 5 s it had run
    assert 5.0 < recs[0]["elapsed_s"] < recs[1]["elapsed_s"]
    # 80 shots in supergathers of 8: 10 encoded forward + adjoint pairs per step
    assert [r["pde_solves_per_sample"] for r in recs] == [60, 80]
    assert not torch.equal(v_half, v_full)  # the last two steps moved the samples
    assert torch.equal(v_res, v_full)
    with pytest.raises(ValueError):
        chains.run_chain(sv, "encoded", 1, eta, seed, nsample=ns, adam_lr=10.0, v0=v0, step0=2)
