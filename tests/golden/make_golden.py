"""Write the stored oracle results used by the full-size GPU parity tests.

Calls only oracle/ (and the seeded input generators).  Run from the
repository root:

    python tests/golden/make_golden.py

gs_fresnel_1024_L8_100it.json -- the 1024x1024 Fresnel, 8-level, 100-iteration
GS workload (target seed 2, phase seed 3, lambda 532 nm, 8 um, z 0.5 m).  For
every SLM state k = 0..100: the SHA-256 of the oracle's level map (uint8,
row-major), the pixels whose quantised angle lies within 1e-5 rad of a level
boundary with the oracle's level there, and nmse[k].
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2006_10509_amd import workloads as wl  # noqa: E402

BAND = 1e-5


def boundary_distance(theta, levels):
    delta = 2 * np.pi / levels
    f = np.mod(np.mod(theta, 2 * np.pi) / delta + 0.5, 1.0)
    return np.minimum(f, 1.0 - f) * delta


def gs_fresnel_1024():
    w = wl.GS_FRESNEL_1024
    t, phi = w.inputs()
    t0 = time.time()
    out = oracle.gs_iterate(t, phi, w.iterations, levels=w.levels,
                            fresnel=dict(wavelength=w.wavelength, pitch=w.pitch, distance=w.distance),
                            trace=True)
    states = []
    for k, st in enumerate(out["trace"]):
        lev = np.ascontiguousarray(st["levels"], dtype=np.uint8)
        dist = boundary_distance(st["angle"], w.levels).ravel()
        band = np.nonzero(dist < BAND)[0]
        states.append({"k": k, "sha256": hashlib.sha256(lev.tobytes()).hexdigest(),
                       "band_index": band.tolist(), "band_level": lev.ravel()[band].tolist()})
    doc = {"workload": w.name, "source": "oracle.gs_iterate (FP64), tests/golden/make_golden.py",
           "band_rad": BAND, "nmse": out["nmse"], "states": states,
           "oracle_seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "gs_fresnel_1024_L8_100it.json"), "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(f"wrote gs_fresnel_1024_L8_100it.json ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    gs_fresnel_1024()
