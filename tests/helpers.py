"""Shared test helpers: the hand-derived golden fixtures."""

import glob
import json
import os

import numpy as np

from paper_1509_06004_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden_instances():
    out = []
    for path in sorted(glob.glob(os.path.join(GOLDEN, "*.json"))):
        with open(path) as f:
            c = json.load(f)
        inst = W.Instance(W=c["W"], H=c["H"], K=c["K"],
                          nlink=np.array(c["nlink"], dtype=np.int32),
                          cap_src=np.array(c["cap_src"], dtype=np.int32),
                          cap_snk0=np.array(c["cap_snk0"], dtype=np.int32),
                          snk_slope=np.array(c["snk_slope"], dtype=np.int32),
                          seed=np.array(c["seed"], dtype=np.uint8),
                          lambdas=np.array(c["lambdas"], dtype=np.int32))
        out.append((c["name"], inst, c["flows"], np.array(c["masks"], dtype=bool)))
    return out
