"""Writes the oracle's values for the full-size workloads to full_size.json.

Run from the repository root:  python tests/golden/make_golden.py [names...]

Every stored value comes from ``oracle/`` (long double Ryser, exact integer
Ryser); the inputs come from the seeded generators, and each entry records the
sha256 of its input so a test can refuse a value whose input drifted.  The
script updates entries in place, so it can be rerun for a subset of names.
"""
import json
import os
import sys
import time
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import default  # noqa: E402
from paper_2502_16577_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "full_size.json")
PARTED = {"u40": 256, "sparse40u": 256}


def inputs():
    return {
        "u20": lambda: W.uniform(20, W.SEED_U20),
        "u32": lambda: W.uniform(32, W.SEED_U32),
        "rademacher32": lambda: W.rademacher(32, W.SEED_RADEMACHER32),
        "haar30": lambda: W.haar_block(120, 30, W.SEED_HAAR120),
        "bernoulli32": lambda: W.bernoulli(32, W.SEED_BERNOULLI32),
        "sparse40": lambda: W.sparse_rows(40, 6, W.SEED_SPARSE40),
        # Table 4 shapes (dense U[0,1), one matrix per order, seed 1000 + n)
        "u35": lambda: W.uniform(35, 1035),
        "u40": lambda: W.uniform(40, 1040),
        # the 40x40 sparse pattern with U[0,1) values (Algorithm 2's CSC walk)
        "sparse40u": lambda: (W.sparse_rows(40, 6, W.SEED_SPARSE40)
                              * W.uniform(40, W.SEED_SPARSE40_VALUES)),
    }


def run_parts(name, a, orc):
    """The unscaled walk in PARTED[name] pieces, resumable; returns the record."""
    nparts = PARTED[name]
    n = int(a.shape[0])
    path = os.path.join(HERE, f"parts_{name}.json")
    state = {"digest": W.digest(a), "nparts": nparts, "parts": {}}
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if old.get("digest") == state["digest"] and old.get("nparts") == nparts:
            state = old
    csc = None
    if name.startswith("sparse"):
        csc = W.to_csc(a)
    for p in range(nparts):
        if str(p) in state["parts"]:
            continue
        t0 = time.time()
        if csc is None:
            (h, l), (ah, al) = orc.ryser_part(a, p, nparts)
        else:
            (h, l), (ah, al) = orc.ryser_part(n, p, nparts, csc=csc)
        state["parts"][str(p)] = [h, l, ah, al, round(time.time() - t0, 2)]
        with open(path + ".tmp", "w") as f:
            json.dump(state, f, indent=0, sort_keys=True)
        os.replace(path + ".tmp", path)
        print(f"{name}: part {p + 1}/{nparts} in {time.time() - t0:.1f} s", flush=True)
    parts = [state["parts"][str(p)] for p in range(nparts)]
    total = sum(Fraction(h) + Fraction(l) for h, l, _, _, _ in parts) * (2 if n % 2 else -2)
    absum = 2 * sum(Fraction(ah) + Fraction(al) for _, _, ah, al, _ in parts)
    hi = float(total)
    lo = float(total - Fraction(hi))
    rec = {"digest": state["digest"], "n": n, "threads": os.cpu_count(), "kind": "real",
           "value": [hi, lo], "abs_sum": float(absum), "abs_perm": hi + lo,
           "oracle_seconds": round(sum(p[4] for p in parts), 2), "parts": nparts}
    if csc is not None:
        rec["oracle"] = "ryser_csc"
    return rec


def run(name, a, orc):
    if name in PARTED:
        return run_parts(name, a, orc)
    t0 = time.time()
    rec = {"digest": W.digest(a), "n": int(a.shape[0]), "threads": os.cpu_count()}
    if a.dtype == np.uint8:
        v, nz = orc.binary(a, with_nonzero=True)
        rec.update(kind="binary", value=str(v), nonzero_terms=nz)
    elif name.startswith("sparse"):
        (h, l), r = orc.sparse(a, with_abs=True, split=True)
        rec.update(kind="real", value=[h, l], abs_sum=r, abs_perm=h + l, oracle="ryser_csc")
    elif np.iscomplexobj(a):
        (rh, rl, ih, il), r = orc.ryser(a, with_abs=True, split=True)
        rec.update(kind="complex", re=[rh, rl], im=[ih, il], abs_sum=r,
                   abs_perm=orc.ryser(np.abs(a)))
    else:
        (h, l), r = orc.ryser(a, with_abs=True, split=True)
        # perm(|A|) is perm(A) itself for a nonnegative matrix (no second sweep)
        ap = h + l if np.all(a >= 0) else orc.ryser(np.abs(a))
        rec.update(kind="real", value=[h, l], abs_sum=r, abs_perm=ap)
    rec["oracle_seconds"] = round(time.time() - t0, 2)
    return rec


def main(names):
    gens = inputs()
    names = names or list(gens)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    orc = default()
    for name in names:
        a = gens[name]()
        rec = run(name, a, orc)
        data[name] = rec
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        print(name, rec, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
