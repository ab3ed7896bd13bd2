"""Parsers for the hand-derived fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def edge_pairs():
    """Rows of tests/golden/edge_pairs.txt as dicts."""
    rows = []
    with open(os.path.join(GOLDEN, "edge_pairs.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, pi, pj, km, note = [t.strip() for t in line.split("|", 4)]
            box, los, n_mu, edges = head.split()
            rows.append(dict(
                box=int(box), los=los, n_mu=int(n_mu),
                edges=np.array([int(e) for e in edges.split(",")], dtype=np.int64),
                pi=np.array([int(v) for v in pi.split()], dtype=np.int64),
                pj=np.array([int(v) for v in pj.split()], dtype=np.int64),
                k=int(km.split()[0]), m=int(km.split()[1]), note=note))
    return rows


def two_point_catalogues(row, scale=1, shift=(0, 0, 0)):
    """The fixture pair as two one-point catalogues (int32 [3, 1] each),
    with coordinates and edges multiplied by ``scale`` and shifted."""
    s = np.asarray(shift, dtype=np.int64)
    a = (row["pi"] * scale + s).reshape(3, 1)
    b = (row["pj"] * scale + s).reshape(3, 1)
    box = row["box"] * scale
    if box:
        a %= box
        b %= box
    return a.astype(np.int32), b.astype(np.int32), row["edges"] * scale, box
