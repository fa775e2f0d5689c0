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


def f32_bits(a):
    """FP32 bit patterns with every NaN as the one quiet NaN 0x7FC00000."""
    b = np.ascontiguousarray(a, np.float32).view(np.uint32).copy()
    b[np.isnan(np.asarray(a, np.float32))] = 0x7FC00000
    return b


# The whole time-frame workload (seed 31): digests of the oracle's tracks, collision times
# and 24-bit compression records, against which the GPU's full-size run is compared bit for
# bit (the oracle needs about two minutes for it, too long for every test run).
TIMEFRAME = ("c3", 31)
Q_STEP = 1.0 / 32.0


def timeframe_summary(cfg=TIMEFRAME[0], seed=TIMEFRAME[1]):
    cs = g.make_config(cfg, seed)
    r = O.Run.from_set(cs)
    K = r.tracks()
    good = K["ndf"] >= 0
    c = O.compress(cs.sector, cs.row, cs.y, cs.z, K, Q_STEP, Q_STEP, wide_z=True)
    return dict(workload=cfg, seed=seed, n_clusters=cs.n,
                input_sha256=digest(np.concatenate([cs.y, cs.z]).view(np.uint32)),
                n_tracks=int(len(K["tracklet"])), n_hits=int(K["off"][-1]),
                track_off_sha256=digest(K["off"]), track_hits_sha256=digest(K["hits"]),
                params_sha256=digest(f32_bits(K["P"][good])), t0_sha256=digest(f32_bits(K["t0"])),
                n_fit_failed=int((~good).sum()), n_t0_nan=int(np.isnan(K["t0"]).sum()),
                cmp_status=int(c["status"]), cmp_n_attached=int(c["n_attached"]),
                cmp_rs_sha256=digest(c["rs"]), cmp_ey_sha256=digest(c["ey"]), cmp_ez_sha256=digest(c["ez"]),
                cmp_ez_hi_sha256=digest(c["ez_hi"]))


if __name__ == "__main__":
    for cfg, seed, scale in CASES:
        out = os.path.join(HERE, f"oracle_{cfg}_seed{seed}.json")
        with open(out, "w") as f:
            json.dump(summary(cfg, seed, scale), f, indent=1)
        print("wrote", out)
    out = os.path.join(HERE, f"oracle_{TIMEFRAME[0]}_seed{TIMEFRAME[1]}_full.json")
    with open(out, "w") as f:
        json.dump(timeframe_summary(), f, indent=1)
    print("wrote", out)
