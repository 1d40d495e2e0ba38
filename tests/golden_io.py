"""Reader for the worked-example fixtures under tests/golden/."""

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_worked_example(name):
    """Returns dict(n=..., ray=(S, P, U, V) float32 arrays, tets=int array, lengths=float array)."""
    n = None
    ray = None
    tets, lens = [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "n":
                n = int(parts[1])
            elif parts[0] == "ray":
                v = np.array([float(x) for x in parts[1:13]], np.float32).reshape(4, 3)
                ray = (v[0], v[1], v[2], v[3])
            else:
                tets.append(int(parts[0]))
                lens.append(float(parts[1]))
    return {"n": n, "ray": ray, "tets": np.array(tets), "lengths": np.array(lens)}
