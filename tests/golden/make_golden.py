"""Writes the stored expected values under tests/golden/ by calling only the oracle (and the seeded
input generators). Run from the repository root:  python -m tests.golden.make_golden
"""
import json
import os

import numpy as np

from fixtures import configs as C
from oracle import scores

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_er_n200():
    w = C.workload(0)
    b = C.build(w)
    gs = scores.batch_scores(b, m=w.m)[0]
    return {
        "workload": w.name,
        "source": "oracle.scores.batch_scores (FP64 Lanczos, CGS2, m=20) on fixtures.configs.workload(0)",
        "m": w.m,
        "K": int(b.K[0]),
        "log_scale": gs.log_scale,
        "scores": gs.s.tolist(),
        "thetas": gs.thetas.tolist(),
        "topk": scores.topk(gs.s, int(b.K[0])).tolist(),
        "targets": sorted(int(x) for x in b.targets[0]),
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "tiny_er_n200_oracle.json"), "w") as f:
        json.dump(tiny_er_n200(), f, indent=1)
    print("wrote", os.path.join(HERE, "tiny_er_n200_oracle.json"))
