"""Writes oracle_regression.json: summaries of the FP64 oracle on fixed seeded
scenes.  Calls only `oracle/` and `lf_scenes/`.

These are regression values of the oracle itself, not values from the paper
(the paper prints none): tests/test_oracle_golden.py recomputes them, so a
change to the oracle's arithmetic shows up as a diff of this file.

    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lf_scenes as S  # noqa: E402
import oracle as O  # noqa: E402

CASES = [
    # (name, workload, overrides, storage, mode, EM iterations)
    ("small-fp32-soft", "small", {}, "f32", "soft", 5),
    ("small-fp16-hard", "small", {"H": 40, "dyn_kind": "ellipse", "dyn_cover": (0.05, 0.4)}, "f16", "hard", 4),
    ("small-bf16-soft-perlin", "small", {"H": 48, "texture": "perlin", "sp_model": "blurflip", "seed": 1777, "dyn_kind": "ellipse", "dyn_cover": (0.05, 0.4)}, "bf16",
     "soft", 3),
]


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def summarize(name, workload, over, storage, mode, n_iters):
    spec = S.workload_spec(workload, **over)
    fr = S.make_frame(spec)
    p = O.make_params(spec.K, spec.H, spec.W, spec.ref, spec.baselines, spec.d_min, spec.d_step, spec.D,
                      fr.beta, gamma=spec.gamma, sigma=spec.sigma, tau=spec.tau, storage=storage, mode=mode)
    r = O.reconstruct(p, fr.views, fr.S_P, fr.mu_T, n_iters)
    return {
        "name": name, "workload": workload, "overrides": over, "storage": storage, "mode": mode, "n_iters": n_iters,
        "inputs_sha256_16": _digest(fr.views) + _digest(fr.S_P) + _digest(fr.mu_T),
        "beta": float(fr.beta),
        "d_idx_histogram": np.bincount(r["d_idx"].ravel(), minlength=spec.D).tolist(),
        "d_idx_sha256_16": _digest(r["d_idx"].astype(np.int32)),
        "L_sum": [float(v) for v in r["L_sum"]],
        "q_sum": float(r["q"].sum()),
        "q_static_count": int((r["q"] >= 0.5).sum()),
        "rho_sum": float(r["rho"].sum()),
        "rgb_sum": float(r["rgb"].sum()),
        "holes": int(r["hole"].sum()),
    }


def main():
    out = [summarize(*c) for c in CASES]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_regression.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
