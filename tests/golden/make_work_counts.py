"""Writes work_counts.json: the exact algorithmic work of the raster on the
benchmark workloads, counted by the oracle (the number of (segment, pixel)
pairs that pass the centre test and the conservative test, Sec. 3.1.2).
These are denominators of the raster's roofline, not expected outputs.

    python tests/golden/make_work_counts.py [head] [lod]
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O                       # noqa: E402
from paper_2607_04230_amd import scenes              # noqa: E402


def counts(name: str) -> dict:
    sc = scenes.build(name)
    table, soff, (ns, ncp) = O.lod_select(sc)
    pos, _, fl = O.generate(sc, table, ncp)
    seg, uc, ua = O.cover_counts(pos, fl, soff, sc.cams, sc.width, sc.height, sc.r_min)
    return {"strands": int(ns), "control_points": int(ncp), "segments": seg,
            "centre_pairs": uc, "conservative_pairs": ua}


def main(names):
    path = os.path.join(HERE, "work_counts.json")
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    for n in names:
        data[n] = counts(n)
        print(n, data[n], flush=True)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["head", "lod"])
