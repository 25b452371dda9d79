"""Writes the oracle regression fixture ``torus512_oracle_hits.csv``.

Calls only the FP64 oracle (``oracle/``) on a seeded subset of the 512-patch
displaced-torus workload (128x128 primary rays + one secondary ray per pixel,
leaf depth 12).  Re-run it only when a change to the oracle's arithmetic is
justified by the paper; the commit that does so names the passage.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1811_03510_amd import scenes as S  # noqa: E402

OUT = os.path.join(HERE, "torus512_oracle_hits.csv")


def rows():
    w = S.config1()
    sc = O.Scene(w.cp, w.types, w.leaf_depth)
    sel_p = S.sample_indices(len(w.primary), 384, seed=101)
    sel_d = S.sample_indices(len(w.diffuse), 256, seed=102)
    out = []
    for cls, rays, sel in (("primary", w.primary, sel_p), ("diffuse", w.diffuse, sel_d)):
        h = sc.intersect(rays[sel], counters=True)
        for k, i in enumerate(sel):
            c = h["counters"][k]
            out.append((cls, int(i), repr(float(h["t"][k])), int(h["id"][k]), repr(float(h["u"][k])),
                        repr(float(h["v"][k])), *[int(x) for x in c]))
    return out


def main():
    with open(OUT, "w") as f:
        f.write("# FP64 oracle hits on a seeded subset of the 512-patch torus workload (L=12).\n")
        f.write("# Written by tests/golden/make_golden.py (calls only oracle/).\n")
        f.write("class,ray,t,patch,u,v," + ",".join(O.COUNTER_NAMES) + "\n")
        for r in rows():
            f.write(",".join(str(x) for x in r) + "\n")
    print(OUT)


if __name__ == "__main__":
    main()
