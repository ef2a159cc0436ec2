"""Reader for the hand-worked fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
INF_I32 = 1 << 30


def _val(tok):
    return INF_I32 if tok == "INF" else int(tok)


def load(name):
    """Returns a dict of named int32 matrices (W/D or A/B/C/OUT)."""
    lines = [l.split("#", 1)[0].strip() for l in open(os.path.join(GOLDEN_DIR, name))]
    lines = [l for l in lines if l]
    out = {}
    i = 0
    n = None
    while i < len(lines):
        parts = lines[i].split()
        key = parts[0]
        if key == "dtype":
            out["dtype"] = parts[1]
            i += 1
        elif key == "n":
            n = int(parts[1])
            i += 1
        elif key in ("W", "D"):
            rows = [[_val(t) for t in lines[i + 1 + r].split()] for r in range(n)]
            out[key] = np.array(rows, dtype=np.int32)
            i += 1 + n
        else:
            r, c = int(parts[1]), int(parts[2])
            rows = [[_val(t) for t in lines[i + 1 + q].split()] for q in range(r)]
            out[key] = np.array(rows, dtype=np.int32).reshape(r, c)
            i += 1 + r
    return out


def fw_fixtures():
    return sorted(f for f in os.listdir(GOLDEN_DIR) if f.startswith("fw_"))
