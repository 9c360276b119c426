"""Storage precision: FP32, shifted FP16 and shifted BF16 population storage against the
FP64 oracle on the two-capsule film box (128 x 128 x 64, two anchored capsules R = 10,
ks = 0.05) after 1000 and 5000 steps, and on the precision-form box (256 x 256 x 96, the
same film and plane, 16 anchored capsules R = 10 at seeded random positions, ks = 0.05)
after 1000, 5000 and 10000 steps.

The reference values are the oracle's, written by tests/golden/make_precision_reference.py.
Measured quantities: meniscus height h(x, y) over the columns where both sides define it
(max and RMS of |dh|, in lattice units), the capillary force on each capsule (relative
error of the vector), and the mass drift of each component relative to its initial mass.

FP32 storage is held to the bounds of the FP32 parity tests.  The 16-bit errors have no
closed form (parity unpinned): they are measured and printed, held to about 1.5 times the
value measured, and a storage that misses the 1 % capillary-force target is reported as an
expected failure (xfail) after those bounds pass.  Each constant-shift 16-bit format runs
with the shift rho_s = rho0 = 1 and without a shift: in this film each
component is 0.7 in one phase and 0.04 in the other, so a shift of 1 leaves the minority
phase stored as -0.96 w_i, and the format's relative precision on that value is a
percent-level error on f_i itself.  The FP16 storage of the relative deviation from each
site's rest equilibrium (``f16site``) stores f_i / (w_i rho_site) - 1, of the order of |u|
in both phases.
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
WORKLOADS = {"c2": dict(ks=0.05), "c3": {}}

# (storage, rho_shift, bounds at the last checkpoint per workload: max |dh|, rms |dh|,
# relative capillary force error, mass drift).  The runs are bitwise deterministic; each
# 16-bit bound is the value measured with the present kernels times about 1.5, so a codec
# change that loses precision fails here.
FP32_BOUNDS = (1e-2, 1e-3, 1e-2, 1e-5)
SANITY = (3.0, 1.5, 5.0, 0.1)
CASES = [
    ("f32", (1.0, 1.0), {"c2": FP32_BOUNDS, "c3": FP32_BOUNDS}),
    ("f16", (1.0, 1.0), {"c2": (1.8, 0.7, 1.8, 3.5e-2), "c3": SANITY}),
    ("f16", (0.0, 0.0), {"c2": (1.1, 0.4, 0.6, 4e-3), "c3": SANITY}),
    ("bf16", (1.0, 1.0), {"c2": (4.0, 0.9, 7.0, 1.5e-2), "c3": SANITY}),
    ("bf16", (0.0, 0.0), {"c2": (3.2, 0.85, 1.4, 1.1e-2), "c3": SANITY}),
    ("f16site", (0.0, 0.0), {"c2": (0.31, 0.05, 0.85, 8.6e-5), "c3": SANITY}),
]
# the accuracy a storage has to reach to stand in for FP32 in the film studies: capillary
# force within 1 % of the FP64 oracle (the force the pair-interaction study measures)
FORCE_TARGET = 1e-2


def _rel(a, b):
    return max(float(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k])) for k in range(len(b)))


def errors(ref, cp, men, caps, mass):
    h0 = ref[f"meniscus_{cp}"].astype(np.float64)
    ok = ~np.isnan(h0) & ~np.isnan(men)
    dh = np.abs(men[ok] - h0[ok])
    fe = _rel(np.array([c["f_capillary"] for c in caps]), ref[f"f_capillary_{cp}"])
    fa = _rel(np.array([c["f_anchor"] for c in caps]), ref[f"f_anchor_{cp}"])
    drift = float(np.max(np.abs(mass - ref["mass0"]) / ref["mass0"]))
    ref_drift = float(np.max(np.abs(ref[f"mass_{cp}"] - ref["mass0"]) / ref["mass0"]))
    return dict(cols=int(ok.sum()), missing=int((np.isnan(h0) != np.isnan(men)).sum()),
                dh_max=float(dh.max()), dh_rms=float(np.sqrt(np.mean(dh * dh))),
                fcap=fe, fanc=fa, drift=drift, ref_drift=ref_drift)


@pytest.mark.parametrize("workload", sorted(WORKLOADS))
@pytest.mark.parametrize("storage,shift,bounds", CASES)
def test_storage_precision_against_oracle(storage, shift, bounds, workload):
    from paper_2007_15405_amd import Sim
    ref_path = os.path.join(GOLDEN, f"{workload}_precision_reference.npz")
    if not os.path.exists(ref_path):
        pytest.skip(f"reference not generated (tests/golden/make_precision_reference.py "
                    f"--workload {workload})")
    ref = np.load(ref_path, allow_pickle=False)
    cfg = synth.workload(workload, **WORKLOADS[workload])
    sim = Sim(cfg, storage=storage, rho_shift=shift)
    m0 = sim.summary()["mass"]
    print(f"\n{workload} {storage} shift {shift}: initial mass rel. to oracle "
          f"{np.max(np.abs(m0 - ref['mass0']) / ref['mass0']):.2e}", flush=True)
    done = 0
    res = {}
    for cp in [int(c) for c in ref["checkpoints"]]:
        sim.step(cp - done)
        done = cp
        obs = sim.observables(meniscus=True, capsules=True)
        res[cp] = errors(ref, cp, obs["meniscus"].astype(np.float64), obs["capsules"],
                         obs["summary"]["mass"])
        r = res[cp]
        print(f"  step {cp}: columns {r['cols']} (definition differs in {r['missing']}), "
              f"max|dh| {r['dh_max']:.3e}, rms|dh| {r['dh_rms']:.3e}, capillary force "
              f"{r['fcap']:.3e}, anchor force {r['fanc']:.3e}, mass drift {r['drift']:.2e} "
              f"(oracle {r['ref_drift']:.1e})", flush=True)
    sim.close()
    hmax, hrms, fcap, drift = bounds[workload]
    r = res[max(res)]
    assert r["dh_max"] <= hmax and r["dh_rms"] <= hrms
    assert r["fcap"] <= fcap
    assert r["drift"] <= drift
    if storage != "f32" and r["fcap"] > FORCE_TARGET:
        pytest.xfail(f"{storage} shift {shift}: capillary force error {r['fcap']:.2e} above "
                     f"the {FORCE_TARGET:.0%} target")
