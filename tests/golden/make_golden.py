"""Writes the oracle regression fixtures in this folder.

Calls only the oracle (and the seeded input generator).  The paper prints no
worked example of the tracking, so these fixtures pin the oracle against
unintended change, not against the paper: the pins of its arithmetic are the
tests in tests/test_oracle_pins.py.  Re-run only together with a change of the
oracle's arithmetic whose commit message names the reading that justifies it.
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle.oracle as O  # noqa: E402
import tpcsynth as g  # noqa: E402

CASES = [("c1", 11, 1.0), ("c2", 21, 0.1)]


def digest(arr):
    return hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()


def summary(cfg, seed, scale):
    cs = g.make_config(cfg, seed, scale=scale)
    r = O.Run.from_set(cs)
    L = r.links()
    T = r.tracklets()
    K = r.tracks()
    return dict(workload=cfg, seed=seed, scale=scale, n_clusters=cs.n,
                input_sha256=digest(np.concatenate([cs.y, cs.z]).view(np.uint32)),
                links_sha256=digest(np.stack([L["up_raw"], L["down_raw"]])),
                n_tracklets=int(len(T["start"])), tracklet_hits_sha256=digest(T["hits"]),
                n_tracks=int(len(K["tracklet"])), track_off_sha256=digest(K["off"]),
                track_hits_sha256=digest(K["hits"]),
                first_params_fp64=K["Pd"][:5].tolist())


if __name__ == "__main__":
    for cfg, seed, scale in CASES:
        out = os.path.join(HERE, f"oracle_{cfg}_seed{seed}.json")
        with open(out, "w") as f:
            json.dump(summary(cfg, seed, scale), f, indent=1)
        print("wrote", out)
