"""Writes the oracle's values for sampled entries of the gradient and
batched workloads to samples.json.

Run from the repository root:  python tests/golden/make_samples.py [names...]

Every stored value comes from ``oracle/`` (long double Ryser, Eq. (1) for
tiny orders, minors and central differences); the inputs come from the
seeded generators, and each entry records the sha256 of its input.

* grad24c / grad24r: the 24 x 24 matrices of the single-matrix gradient
  row (a 120 x 120 Haar block; U[0,1) seed 1024): the permanent, R(A),
  perm(|A|), and minors at fixed positions with their perm(|minor|).
* batched: the 4096-matrix photon-counting batch (orders 8..24).  A seeded
  sample of 256 (m, i, j) minors and 256 (m, i, j) central differences over
  matrices of order 13..24, a quarter of each from every band of orders
  (13-16, 17-20, 21-22, 23-24), and the permanents (with R(A) and
  perm(|A|)) of 40 seeded matrices of orders 21..24 and 24 of orders 8..20.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import default  # noqa: E402
from paper_2502_16577_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "samples.json")
GRAD_POSITIONS = [(0, 0), (3, 17), (11, 5), (23, 23), (17, 0), (8, 12)]
BANDS = [(13, 16), (17, 20), (21, 22), (23, 24)]


def cplx(z):
    return [float(np.real(z)), float(np.imag(z))]


def minor_of(a, i, j):
    return np.delete(np.delete(a, i, 0), j, 1)


def grad_entry(a, orc):
    rec = {"digest": W.digest(a), "n": int(a.shape[0])}
    v, r = orc.ryser(a, with_abs=True)
    rec.update(perm=cplx(v), abs_sum=r, abs_perm=float(np.real(orc.ryser(np.abs(a)))))
    rec["minors"] = []
    for i, j in GRAD_POSITIONS:
        m = minor_of(a, i, j)
        rec["minors"].append({"i": i, "j": j, "value": cplx(orc.ryser(m)),
                              "abs_perm": float(np.real(orc.ryser(np.abs(m))))})
    return rec


def batched_entry(orc):
    mats = W.batched_submatrices(4096, 8, 24)
    ks, offs, data = W.pack(mats)
    rec = {"digest": W.digest(data), "count": 4096}
    rng = np.random.default_rng(20250216)
    by_band = [[m for m in range(4096) if lo <= mats[m].shape[0] <= hi] for lo, hi in BANDS]

    def triples(count):
        out = []
        for band in by_band:
            for _ in range(count // len(BANDS)):
                m = int(rng.choice(band))
                k = mats[m].shape[0]
                out.append((m, int(rng.integers(k)), int(rng.integers(k))))
        return out

    rec["minors"] = []
    for m, i, j in triples(256):
        a = mats[m]
        sub = minor_of(a, i, j)
        rec["minors"].append({"m": m, "k": int(a.shape[0]), "i": i, "j": j,
                              "value": cplx(orc.perm(sub)),
                              "abs_perm": float(np.real(orc.perm(np.abs(sub))))})
    rec["fd"] = []
    for m, i, j in triples(256):
        a = mats[m]
        rec["fd"].append({"m": m, "k": int(a.shape[0]), "i": i, "j": j, "h": 0.125,
                          "value": cplx(orc.grad_fd(a, i, j, h=0.125))})
    rec["perms"] = []
    big = [m for m in range(4096) if mats[m].shape[0] >= 21]
    small = [m for m in range(4096) if mats[m].shape[0] <= 20]
    for m in list(rng.choice(big, size=40, replace=False)) + list(rng.choice(small, size=24, replace=False)):
        a = mats[int(m)]
        v, r = orc.ryser(a, with_abs=True)
        rec["perms"].append({"m": int(m), "k": int(a.shape[0]), "value": cplx(v), "abs_sum": r,
                             "abs_perm": float(np.real(orc.ryser(np.abs(a))))})
    return rec


def inputs():
    return {
        "grad24c": lambda orc: grad_entry(W.haar_block(120, 24, W.SEED_HAAR120), orc),
        "grad24r": lambda orc: grad_entry(W.uniform(24, 1024), orc),
        "batched": batched_entry,
    }


def main(names):
    gens = inputs()
    names = names or list(gens)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    orc = default()
    for name in names:
        t0 = time.time()
        rec = gens[name](orc)
        rec["oracle_seconds"] = round(time.time() - t0, 2)
        rec["threads"] = os.cpu_count()
        data[name] = rec
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        print(name, rec["oracle_seconds"], "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
