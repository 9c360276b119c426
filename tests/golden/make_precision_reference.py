"""FP64 oracle reference for the storage-precision study.

Workloads:
* ``c2``: the film-drying box of two anchored capsules (128 x 128 x 64 lattice, wall at
  z = 0, film 12 layers high, repulsive plane 10 lattice units above the wall, capsules
  R = 10 of 5120 triangles at separation 3R, ks = 0.05, anchor spring 1), checkpoints
  1000 and 5000 steps;
* ``c3``: the precision form's box (256 x 256 x 96, the same film and plane, 16 anchored
  capsules R = 10 at seeded random positions, ks = 0.05), checkpoints 1000, 5000 and
  10000 steps.
The oracle is stepped to each checkpoint and its meniscus height field, capsule
observables and component masses are written to ``<workload>_precision_reference.npz``
next to this script.

``--precision f32 --until N`` runs the oracle's FP32 build instead, to the checkpoints up
to N, and writes ``<workload>_precision_oracle_f32.npz``: the same quantities from an
independent FP32 computation, which bound how far FP32 arithmetic alone moves them from
the FP64 reference.

Only the oracle and the seeded input generators are used.  Run from the repository root:

    python tests/golden/make_precision_reference.py [--workload c2|c3] [--threads N]
        [--precision f64|f32] [--until STEPS]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

CHECKPOINTS = {"c2": (1000, 5000), "c3": (1000, 5000, 10000)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--workload", default="c2", choices=sorted(CHECKPOINTS))
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--until", type=int, default=0)
    args = ap.parse_args()
    cfg = synth.workload("c2", ks=0.05) if args.workload == "c2" else synth.workload("c3")
    name = "reference" if args.precision == "f64" else "oracle_f32"
    out = os.path.join(HERE, f"{args.workload}_precision_{name}.npz")
    cps = [c for c in CHECKPOINTS[args.workload] if args.until <= 0 or c <= args.until]
    o = oracle.Oracle(cfg, args.precision, n_threads=args.threads)
    ncap = len(cfg["capsules"])
    mass0 = o.summary()["mass"].copy()
    rec = dict(checkpoints=np.array(cps), mass0=mass0)
    done = 0
    t0 = time.time()
    for cp in cps:
        st = o.step(cp - done)
        if st != 0:
            raise SystemExit(f"oracle step failed with status {st}")
        done = cp
        caps = [o.capsule(k) for k in range(ncap)]
        rec[f"meniscus_{cp}"] = o.meniscus().astype(np.float32)
        rec[f"mass_{cp}"] = o.summary()["mass"].copy()
        for key in ("centroid", "f_capillary", "f_anchor", "f_hertz"):
            rec[f"{key}_{cp}"] = np.array([c[key] for c in caps])
        rec[f"volume_{cp}"] = np.array([c["volume"] for c in caps])
        print(f"step {cp}: {time.time() - t0:.0f} s", flush=True)
    o.close()
    np.savez_compressed(out, **rec)
    print("wrote", out)


if __name__ == "__main__":
    main()
