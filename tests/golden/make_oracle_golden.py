"""Write oracle_tiny_2d.json: the FP64 oracle's data, misfits and gradient for a tiny
encoded 2D problem (two supergathers of one sample, +-1 weights), the stored expectation
that tests/test_golden.py (oracle regression) and tests/test_gpu_parity.py (HIP path)
compare against.  Calls only the oracle and the seeded input generators.

Run from the repository root:  python tests/golden/make_oracle_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

PROBLEM = {
    "grid": {"nz": 20, "nx": 30, "dz": 10.0, "dx": 10.0, "nb": 5, "v_ref": 3000.0},
    "dt": 1e-3, "nt": 200, "rec_every": 2,
    "model": {"kind": "linear_gradient", "top": 1800.0, "bottom": 2800.0},
    "truth_scale": 0.9,
    "wavelet": {"kind": "ricker", "freq": 25.0},
    "sims": [{"src": [[1, 5], [1, 15], [1, 25]], "w": [1.0, -1.0, 1.0]},
             {"src": [[1, 10], [1, 20]], "w": [-1.0, 1.0]}],
    "receivers": {"row": 1, "every": 2},
    "inv_sigma2": 1.0,
}


def build_problem(p=PROBLEM):
    """(oracle grid, FP32-rounded model, truth, wavelet, [(cells, weights)], receivers)."""
    g = p["grid"]
    grid = oracle.Grid(nz=g["nz"], nx=g["nx"], dz=g["dz"], dx=g["dx"], nb=g["nb"], v_ref=g["v_ref"])
    v = W.linear_gradient(g["nz"], g["nx"], p["model"]["top"], p["model"]["bottom"])
    v = np.asarray(v, dtype=np.float32).astype(np.float64).ravel()
    truth = (np.asarray(v * p["truth_scale"], dtype=np.float32)).astype(np.float64)
    wav = np.asarray(W.ricker(p["wavelet"]["freq"], p["dt"], p["nt"]), dtype=np.float32)
    sims = [(np.array([z * g["nx"] + x for z, x in s["src"]], dtype=np.int32), np.array(s["w"], dtype=np.float32))
            for s in p["sims"]]
    rec = np.array([p["receivers"]["row"] * g["nx"] + x for x in range(0, g["nx"], p["receivers"]["every"])],
                   dtype=np.int32)
    return grid, v, truth, wav, sims, rec


def observed(p=PROBLEM):
    """Observed data of each supergather: exact-coefficient forward on the 10 % slower
    truth, rounded to FP32 (the precision the library receives)."""
    grid, v, truth, wav, sims, rec = build_problem(p)
    return [oracle.forward(grid, truth, p["dt"], p["nt"], p["rec_every"], c, w, wav, rec,
                           coef_fp32=False).astype(np.float32).astype(np.float64) for c, w in sims]


def sample_points(d, k=12):
    """(t, r) of the k largest-magnitude entries of d, in row-major order."""
    idx = np.sort(np.argsort(np.abs(d).ravel(), kind="stable")[-k:])
    return [[int(i // d.shape[1]), int(i % d.shape[1])] for i in idx]


def compute(p=PROBLEM):
    grid, v, truth, wav, sims, rec = build_problem(p)
    out = {"misfit": [], "d_pred_norm": [], "d_pred_samples": [], "gradient": None}
    gsum = np.zeros(grid.nphys)
    for (cells, w), d_obs in zip(sims, observed(p)):
        d, phi, g = oracle.gradient(grid, v, p["dt"], p["nt"], p["rec_every"], cells, w, wav, rec, d_obs,
                                    p["inv_sigma2"], coef_fp32=True)
        out["misfit"].append(phi)
        out["d_pred_norm"].append(float(np.linalg.norm(d)))
        out["d_pred_samples"].append([[t, r, float(d[t, r])] for t, r in sample_points(d)])
        gsum += g
    out["gradient"] = [float("%.17g" % x) for x in gsum]  # the sample's gradient, kappa = 1
    return out


if __name__ == "__main__":
    res = compute()
    res["problem"] = PROBLEM
    res["about"] = ("FP64 oracle (FP32-rounded coefficient set) on a tiny 2D problem: 20 x 30 grid, 5-cell "
                    "sponge, 200 steps, one sample with two +-1 supergathers; written by make_oracle_golden.py")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_tiny_2d.json")
    with open(path, "w") as f:
        json.dump(res, f)
    print("wrote", path, os.path.getsize(path), "bytes")
