"""Writes tests/golden/oracle_regression.json from the CPU oracle only.

These stored values pin the oracle against unintended changes of its
arithmetic: any later change that alters them must name, in its commit
message, the passage of the paper (or the reading of it) that justifies it.
Run: python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from netgen import configs  # noqa: E402
from oracle import Oracle  # noqa: E402


def digest(spec, steps, prec):
    o = Oracle(spec, prec)
    o.step(steps)
    st, ids = o.spikes()
    V, J, ref = o.state()
    h = hashlib.sha256()
    h.update(st.astype("<u8").tobytes())
    h.update(ids.astype("<u4").tobytes())
    hs = hashlib.sha256()
    hs.update(V.astype("<f8").tobytes())
    hs.update(J.astype("<f8").tobytes())
    hs.update(ref.astype("<i4").tobytes())
    return {"steps": steps, "precision": prec, "spikes": int(len(st)), "edge_events": o.edge_events,
            "raster_sha256": h.hexdigest(), "state_sha256": hs.hexdigest()}


CASES = {
    "tiny_1s_fp32": (lambda: configs.tiny(), 10000, 32),
    "tiny_200ms_fp64": (lambda: configs.tiny(), 2000, 64),
    "share_3000_k100_50ms_fp32": (lambda: configs.share(n=3000, indegree=100, bg_rate_hz=7000.0, seed=2), 500, 32),
    "regions_6x100_50ms_fp32": (lambda: configs.multi_region(n_regions=6, per_region=100, intra_indegree=40,
                                                             long_indegree=10, seed=1, bg_rate_hz=5600.0),
                                500, 32),
}

if __name__ == "__main__":
    out = {name: digest(f(), steps, prec) for name, (f, steps, prec) in CASES.items()}
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))
