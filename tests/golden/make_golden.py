"""Write the stored oracle results used by the full-size GPU parity tests.

Calls only oracle/ (and the seeded input generators).  Run from the
repository root:

    python tests/golden/make_golden.py [gs] [ospr] [pairs]     (default: all)

gs_fresnel_1024_L8_100it.json -- the 1024x1024 Fresnel, 8-level, 100-iteration
GS workload (target seed 2, phase seed 3, lambda 532 nm, 8 um, z 0.5 m).  For
every SLM state k = 0..100: the SHA-256 of the oracle's level map (uint8,
row-major), the pixels whose quantised angle lies within 1e-5 rad of a level
boundary with the oracle's level there, and nmse[k].

ospr_2048_24sub.json -- the 2048x2048 binary OSPR workload, 24 subframes
(target seed 4, subframe phase seeds 10..33).  For every subframe: the pixels
whose sign decision lies in the boundary band |Re G| < 1e-5 |G| with the
oracle's level there, and the SHA-256 of the oracle's level map (uint8,
row-major) with those pixels set to 255; then the NMSE of the averaged
intensity, its sum, its 64 x 64 grid of 32 x 32 block sums and its value at
4096 pixels drawn from default_rng(2048).

ospr_pairs_2048_12pairs.json -- the same workload as 12 real/imaginary pairs
(subframe phase seeds 10..21; subframe 2n from Re G_n, 2n + 1 from Im G_n),
stored the same way (band |Re G| or |Im G| < 1e-5 |G|).
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


def masked_sha(lev, band_index):
    flat = np.ascontiguousarray(lev, dtype=np.uint8).ravel().copy()
    flat[band_index] = 255
    return hashlib.sha256(flat.tobytes()).hexdigest()


def intensity_summary(avg, nmse):
    h, w = avg.shape
    blocks = avg.reshape(64, h // 64, 64, w // 64).sum(axis=(1, 3))
    rng = np.random.default_rng(2048)
    idx = np.sort(rng.choice(h * w, size=4096, replace=False))
    return {"nmse": float(nmse), "sum": float(avg.sum()),
            "block_sums_64x64": [float(f"{v:.12e}") for v in blocks.ravel()],
            "sample_index": idx.tolist(), "sample_value": [float(f"{v:.12e}") for v in avg.ravel()[idx]]}


def ospr_2048(pairs=False):
    w = wl.OSPR_2048
    t = w.target().astype(np.float64)
    n_in = w.subframes // 2 if pairs else w.subframes
    thetas = w.subframe_phases(n_in)
    t0 = time.time()
    out = (oracle.ospr_pairs if pairs else oracle.ospr)(t, thetas)
    subframes = []
    for n in range(n_in):
        g = oracle.ifft2(oracle.ifftshift(t * np.exp(1j * thetas[n].astype(np.float64))))
        parts = (g.real, g.imag) if pairs else (g.real,)
        for k, part in enumerate(parts):
            m = len(parts) * n + k
            band = np.nonzero((np.abs(part) < BAND * np.abs(g)).ravel())[0]
            lev = out["levels"][m]
            subframes.append({"n": m, "band_index": band.tolist(), "band_level": lev.ravel()[band].tolist(),
                              "masked_sha256": masked_sha(lev, band)})
    name = "ospr_pairs_2048_12pairs.json" if pairs else "ospr_2048_24sub.json"
    doc = {"workload": w.name + ("_pairs" if pairs else ""),
           "source": f"oracle.{'ospr_pairs' if pairs else 'ospr'} (FP64), tests/golden/make_golden.py",
           "band_rel": BAND, "subframes": subframes, **intensity_summary(out["intensity"], out["nmse"]),
           "oracle_seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(f"wrote {name} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    which = sys.argv[1:] or ["gs", "ospr", "pairs"]
    if "gs" in which:
        gs_fresnel_1024()
    if "ospr" in which:
        ospr_2048()
    if "pairs" in which:
        ospr_2048(pairs=True)
