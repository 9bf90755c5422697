"""Writes tests/golden/oracle_digests.json: sha256 digests of the CPU oracle's
diagrams of the full-size workloads.  Calls only oracle/ and synth (the input
generators); nothing from the GPU path.

Each entry records the digest of the float32 input bytes and of the diagram
bytes (dim int32, birth float32, death float32, birth_pixel int64, death_pixel
int64, concatenated, canonical row order, pixel indices local to the image) and
the number of rows per dimension.  Run: python tests/golden/make_oracle_digests.py
[NAME ...] (with names, only those entries are computed and merged into the
existing file).
"""
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_digests.json")


def input_digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, np.float32).tobytes()).hexdigest()


def diagram_digest(dim, birth, death, bp, dp) -> str:
    h = hashlib.sha256()
    for arr, dt in ((dim, np.int32), (birth, np.float32), (death, np.float32), (bp, np.int64), (dp, np.int64)):
        h.update(np.ascontiguousarray(arr, dt).tobytes())
    return h.hexdigest()


def entry(img):
    d = oracle.persistence(img)
    return {"input": input_digest(img), "diagram": diagram_digest(d.dim, d.birth, d.death, d.birth_pixel,
                                                                 d.death_pixel),
            "rows_per_dim": np.bincount(d.dim, minlength=3).tolist()}


def masked_c3():
    """The 256^3 volume with +inf outside the inscribed ball."""
    v = synth.config("C3")
    return np.where(synth.ball_mask(v.shape), v, np.float32(np.inf)).astype(np.float32)


def walk_2_24():
    return synth.random_walk(1 << 24)


EXTRA = {"C3_masked": masked_c3, "walk_2_24": walk_2_24}


def main():
    if len(sys.argv) > 1:
        out = json.load(open(OUT))
        t = time.time()
        for name in sys.argv[1:]:
            out[name] = entry(EXTRA[name]())
            print(f"{name}: {time.time() - t:.0f} s", flush=True)
        json.dump(out, open(OUT, "w"), indent=1)
        return
    out = {}
    t = time.time()
    with cf.ThreadPoolExecutor(8) as ex:
        c4 = ex.submit(lambda: list(ex.map(entry, synth.config("C4"))))
        c5 = ex.submit(lambda: list(ex.map(entry, synth.config("C5"))))
        out["C3"] = entry(synth.config("C3"))
        out["C4"] = c4.result()
        out["C5"] = c5.result()
    out["C2"] = entry(synth.config("C2"))
    for name, make in EXTRA.items():
        out[name] = entry(make())
    json.dump(out, open(OUT, "w"), indent=1)
    print(f"wrote {OUT} in {time.time() - t:.0f} s")


if __name__ == "__main__":
    main()
