"""Reader for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def closed_forms():
    """List of dicts {name, k, why, image (uint8 HxW), codes (uint8 hxw)}."""
    cases = []
    with open(os.path.join(GOLDEN, "closed_forms.txt")) as f:
        lines = [ln.rstrip("\n") for ln in f if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        assert lines[i].startswith("case "), lines[i]
        c = {"name": lines[i][5:]}
        c["k"] = int(lines[i + 1].split()[1])
        c["why"] = lines[i + 2][4:]
        _, H, W = lines[i + 3].split()
        H, W = int(H), int(W)
        c["image"] = np.array([[int(v) for v in lines[i + 4 + r].split()] for r in range(H)],
                              dtype=np.uint8)
        j = i + 4 + H
        _, h, w = lines[j].split()
        h, w = int(h), int(w)
        c["codes"] = np.array([[int(v) for v in lines[j + 1 + r].split()] for r in range(h)],
                              dtype=np.uint8)
        cases.append(c)
        i = j + 1 + h
    return cases
