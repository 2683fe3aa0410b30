"""SHA-256 digests of oracle outputs for frames too large to run the oracle
inside a GPU test (the 1920x1080 / D=256 frame alone takes about 35 s of
single-threaded oracle time).

    python tests/golden/oracle_digests.py        # rewrites oracle_digests.json

The digests are written by this script from ``oracle`` alone (plain C, single
thread) on the seeded inputs of ``paper_2106_07927_amd.datagen``; nothing here
calls the HIP path.  Each case also records the digests of its two input
images, so a GPU test can tell "the generator changed" apart from "the
results differ".

Cases (all with census 9x7, 8 paths, P1 = 10, P2 = 120, LR tolerance 1,
3x3 median):
  * the 1920x1080 / D=256 frame: every intermediate (census of both images,
    cost, S_bar, D^L, D^R) and the final map;
  * one pair per distinct (W, H, D) of the 64-pair mixed batch (its first
    occurrence in the batch, the batch's noise images): D and D^R;
  * two frames per distinct (W, H, D) of the 16 served camera streams (the
    first stream of each shape, frames 0 and 1 of its pool): D.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

JSON_PATH = os.path.join(HERE, "oracle_digests.json")
PARAMS = dict(win_w=9, win_h=7, npaths=8, p1=10, p2=120, lr_tolerance=1, median3x3=True)
SERVE_FRAMES = 2


def digest(a) -> str:
    """Digest of an array's dtype, shape and C-order bytes."""
    a = np.ascontiguousarray(a)
    h = hashlib.sha256()
    h.update(f"{a.dtype.str}{a.shape}".encode())
    h.update(a.tobytes())
    return h.hexdigest()


def cases():
    """(name, spec) of every case; spec says how to draw the inputs."""
    from paper_2106_07927_amd import datagen
    out = [("c3_1920x1080_d256_r8", {"kind": "config", "config": "c3_1920x1080_d256_r8",
                                      "ndisp": 256, "outputs": ["census_left", "census_right",
                                                                "cost", "agg", "disp_left",
                                                                "disp_right", "disp"]})]
    seen = set()
    for (w, h, nd, seed) in datagen.batch_specs():
        if (w, h, nd) in seen:
            continue
        seen.add((w, h, nd))
        out.append((f"batch_{w}x{h}x{nd}", {"kind": "noise", "width": w, "height": h, "ndisp": nd,
                                            "seed": seed, "outputs": ["disp", "disp_right"]}))
    seen = set()
    for (w, h, nd, seed) in datagen.stream_specs():
        if (w, h, nd) in seen:
            continue
        seen.add((w, h, nd))
        for k in range(SERVE_FRAMES):
            out.append((f"serve_{w}x{h}x{nd}_{k}",
                        {"kind": "stream", "width": w, "height": h, "ndisp": nd,
                         "stream_seed": seed, "frame": k, "outputs": ["disp"]}))
    return sorted(out)


def case_inputs(spec):
    """(left, right) uint8 images of a case, from the seeded generator."""
    from paper_2106_07927_amd import datagen
    if spec["kind"] == "config":
        pair = datagen.config_pair(spec["config"])
        return pair["left"], pair["right"]
    if spec["kind"] == "noise":
        return datagen.random_images(spec["width"], spec["height"], spec["seed"])
    pair = datagen.make_pair(spec["width"], spec["height"], spec["ndisp"],
                             spec["stream_seed"] * 10 + spec["frame"], (8, 16), 0.05)
    return pair["left"], pair["right"]


def stream_frame_case(width, height, ndisp, stream_seed, frame):
    """Name of the served-frame case for a stream of this shape and seed, or
    None when it is not a stored case."""
    for name, spec in cases():
        if spec["kind"] == "stream" and (spec["width"], spec["height"], spec["ndisp"],
                                         spec["stream_seed"], spec["frame"]) == \
                (width, height, ndisp, stream_seed, frame):
            return name
    return None


def load():
    with open(JSON_PATH) as f:
        return json.load(f)


def main():
    import oracle
    table = {"params": PARAMS, "cases": {}}
    for name, spec in cases():
        t0 = time.perf_counter()
        left, right = case_inputs(spec)
        ref = oracle.run(left, right, oracle.Params(ndisp=spec["ndisp"], **PARAMS))
        table["cases"][name] = {
            "spec": spec,
            "inputs": {"left": digest(left), "right": digest(right)},
            "outputs": {k: digest(ref[k]) for k in spec["outputs"]},
        }
        print(f"{name}: {time.perf_counter() - t0:.1f} s", flush=True)
    with open(JSON_PATH, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
