"""Write the oracle's values on the evaluation sets of the two full-size configurations.

For the 2048^2 spherical cap and the 4096^2 sinusoidal relief (``synth.config``
names ``cap_2048`` and ``sinusoid_4096``) the evaluation sets are a 256^2 centre
crop [M/2 - 128, M/2 + 128)^2, a 256^2 corner crop [M - 256, M)^2 (the largest
|m|, |n|, where the deconvolution divides by the smallest kernel transform) and
4096 random pixels (``synth.sample_pixels`` seed 1).  The crops come from
``oracle.crop_gemm``, the random pixels from ``oracle.direct``; nothing here
runs or reads the GPU path.  Each file records a SHA-256 of the inputs it was
computed from, which the tests check before comparing.

Usage (repository root):  python tests/golden/make_eval_sets.py [cap_2048] [sinusoid_4096]
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CROP = 256
N_RANDOM = 4096
RANDOM_SEED = 1
CONFIGS = ("cap_2048", "sinusoid_4096")


def input_digest(w) -> str:
    """SHA-256 of a workload's arrays and optics (what the stored values depend on)."""
    h = hashlib.sha256()
    for a in (w.x, w.y, w.d, w.u):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(repr((w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my, w.incident)).encode())
    return h.hexdigest()


def eval_set_ranges(w):
    """(centre (ix range, iy range), corner (ix range, iy range), random (ix, iy))."""
    import synth

    cx, cy = w.mx // 2 - CROP // 2, w.my // 2 - CROP // 2
    centre = (range(cx, cx + CROP), range(cy, cy + CROP))
    corner = (range(w.mx - CROP, w.mx), range(w.my - CROP, w.my))
    rand = synth.sample_pixels(w.mx, w.my, N_RANDOM, seed=RANDOM_SEED)
    return centre, corner, rand


def path_for(name: str) -> str:
    return os.path.join(HERE, f"eval_sets_{name}.npz")


def make(name: str) -> str:
    import oracle
    import synth

    w = synth.config(name)
    centre, corner, (rix, riy) = eval_set_ranges(w)
    t0 = time.time()
    args = (w.x, w.y, w.d, w.u, w.lam, w.z0, w.p2x, w.p2y, w.mx, w.my)
    v_centre = oracle.crop_gemm(*args, centre[0], centre[1], incident=w.incident)
    v_corner = oracle.crop_gemm(*args, corner[0], corner[1], incident=w.incident)
    t1 = time.time()
    v_rand = oracle.direct(*args, rix, riy, incident=w.incident)
    t2 = time.time()
    out = path_for(name)
    np.savez(out, config=name, digest=input_digest(w),
             centre_x0=centre[0].start, centre_y0=centre[1].start,
             corner_x0=corner[0].start, corner_y0=corner[1].start, crop=CROP,
             centre=v_centre, corner=v_corner, random_ix=rix, random_iy=riy, random=v_rand)
    print(f"{name}: crops {t1 - t0:.1f} s (crop_gemm), {len(rix)} random pixels {t2 - t1:.1f} s (direct) -> {out}")
    return out


def load(name: str):
    """The stored sets as {set: (ix, iy, values)} (flat arrays) and the stored input digest."""
    z = np.load(path_for(name), allow_pickle=False)
    sets = {}
    for s in ("centre", "corner"):
        x0, y0, c = int(z[f"{s}_x0"]), int(z[f"{s}_y0"]), int(z["crop"])
        gx, gy = np.meshgrid(np.arange(x0, x0 + c), np.arange(y0, y0 + c))
        sets[s] = (gx.reshape(-1), gy.reshape(-1), z[s].reshape(-1))
    sets["random"] = (z["random_ix"], z["random_iy"], z["random"])
    return sets, str(z["digest"])


if __name__ == "__main__":
    for nm in (sys.argv[1:] or CONFIGS):
        if nm not in CONFIGS:
            raise SystemExit(f"unknown configuration {nm!r}; choose from {CONFIGS}")
        make(nm)
