"""Loader for the hand-derived fixtures in tests/golden/."""
import glob
import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(path):
    scale = None
    pts, expect = [], None
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "scale":
                scale = int(tok[1])
            elif tok[0] == "p":
                pts.append((int(tok[1]), int(tok[2])))
            elif tok[0] == "expect":
                expect = [int(t) for t in tok[1:]]
    assert scale and (scale & (scale - 1)) == 0
    xy = np.array(pts, dtype=np.float64) / scale
    return xy.astype(np.float32), np.array(expect, dtype=np.int32)


def all_fixtures():
    return sorted(glob.glob(os.path.join(GOLDEN_DIR, "*.txt")))
