"""Regression of the oracle against its stored fixture (see tests/golden/make_golden.py)."""
import os

import numpy as np

import oracle as O

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_matches_stored_fixture(c1, c1_oracle):
    import csv
    with open(os.path.join(HERE, "torus512_oracle_hits.csv")) as f:
        rows = [r for r in csv.reader(line for line in f if not line.startswith("#"))]
    header, rows = rows[0], rows[1:]
    assert header[:6] == ["class", "ray", "t", "patch", "u", "v"]
    for cls in ("primary", "diffuse"):
        sub = [r for r in rows if r[0] == cls]
        idx = np.array([int(r[1]) for r in sub])
        rays = (c1.primary if cls == "primary" else c1.diffuse)[idx]
        h = c1_oracle.intersect(rays, counters=True)
        np.testing.assert_array_equal(h["t"], np.array([float(r[2]) for r in sub]))
        np.testing.assert_array_equal(h["id"], np.array([int(r[3]) for r in sub], np.uint32))
        np.testing.assert_array_equal(h["u"], np.array([float(r[4]) for r in sub]))
        np.testing.assert_array_equal(h["v"], np.array([float(r[5]) for r in sub]))
        np.testing.assert_array_equal(h["counters"], np.array([[int(x) for x in r[6:14]] for r in sub]))
