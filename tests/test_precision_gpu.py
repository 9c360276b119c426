"""Storage precision: FP32, shifted FP16 and shifted BF16 population storage against the
FP64 oracle on the two-capsule film box (128 x 128 x 64, two anchored capsules R = 10,
ks = 0.05), after 1000 and 5000 steps.

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
percent-level error on f_i itself.  The FP16 storage shifted by each site's own density
(``f16site``) stores only f_i - w_i rho_site, of the order of w_i rho |u|.
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

REF = os.path.join(os.path.dirname(__file__), "golden", "c2_precision_reference.npz")

# (storage, rho_shift, bounds at 5000 steps: max |dh|, rms |dh|, relative capillary force
# error, mass drift).  The runs are bitwise deterministic; each 16-bit bound is the value
# measured with the present kernels times about 1.5, so a codec change that loses
# precision fails here.
FP32_BOUNDS = (1e-2, 1e-3, 1e-2, 1e-5)
CASES = [
    ("f32", (1.0, 1.0), FP32_BOUNDS),
    ("f16", (1.0, 1.0), (1.8, 0.7, 1.8, 3.5e-2)),
    ("f16", (0.0, 0.0), (1.1, 0.4, 0.6, 4e-3)),
    ("bf16", (1.0, 1.0), (4.0, 0.9, 7.0, 1.5e-2)),
    ("bf16", (0.0, 0.0), (3.2, 0.85, 1.4, 1.1e-2)),
    ("f16site", (0.0, 0.0), (3.0, 1.5, 5.0, 0.1)),
]
# the accuracy a storage has to reach to stand in for FP32 in the film studies: capillary
# force within 1 % of the FP64 oracle (the force the pair-interaction study measures)
FORCE_TARGET = 1e-2

def errors(ref, cp, men, caps, mass):
    h0 = ref[f"meniscus_{cp}"].astype(np.float64)
    ok = ~np.isnan(h0) & ~np.isnan(men)
    dh = np.abs(men[ok] - h0[ok])
    fr = ref[f"f_capillary_{cp}"]
    fe = max(float(np.linalg.norm(caps[k] - fr[k]) / np.linalg.norm(fr[k])) for k in range(len(fr)))
    drift = float(np.max(np.abs(mass - ref["mass0"]) / ref["mass0"]))
    ref_drift = float(np.max(np.abs(ref[f"mass_{cp}"] - ref["mass0"]) / ref["mass0"]))
    return dict(cols=int(ok.sum()), missing=int((np.isnan(h0) != np.isnan(men)).sum()),
                dh_max=float(dh.max()), dh_rms=float(np.sqrt(np.mean(dh * dh))),
                fcap=fe, drift=drift, ref_drift=ref_drift)


@pytest.mark.parametrize("storage,shift,bounds", CASES)
def test_storage_precision_against_oracle(storage, shift, bounds):
    from paper_2007_15405_amd import Sim
    if not os.path.exists(REF):
        pytest.skip("reference not generated (tests/golden/make_precision_reference.py)")
    ref = np.load(REF, allow_pickle=False)
    cfg = synth.workload("c2", ks=0.05)
    sim = Sim(cfg, storage=storage, rho_shift=shift)
    m0 = sim.summary()["mass"]
    print(f"\n{storage} shift {shift}: initial mass rel. to oracle "
          f"{np.max(np.abs(m0 - ref['mass0']) / ref['mass0']):.2e}", flush=True)
    done = 0
    res = {}
    for cp in [int(c) for c in ref["checkpoints"]]:
        sim.step(cp - done)
        done = cp
        obs = sim.observables(meniscus=True, capsules=True)
        caps = [c["f_capillary"] for c in obs["capsules"]]
        res[cp] = errors(ref, cp, obs["meniscus"].astype(np.float64), caps, obs["summary"]["mass"])
        r = res[cp]
        print(f"  step {cp}: columns {r['cols']} (definition differs in {r['missing']}), "
              f"max|dh| {r['dh_max']:.3e}, rms|dh| {r['dh_rms']:.3e}, capillary force "
              f"{r['fcap']:.3e}, mass drift {r['drift']:.2e} (oracle {r['ref_drift']:.1e})",
              flush=True)
    sim.close()
    hmax, hrms, fcap, drift = bounds
    r = res[max(res)]
    assert r["dh_max"] <= hmax and r["dh_rms"] <= hrms
    assert r["fcap"] <= fcap
    assert r["drift"] <= drift
    if storage != "f32" and r["fcap"] > FORCE_TARGET:
        pytest.xfail(f"{storage} shift {shift}: capillary force error {r['fcap']:.2e} above "
                     f"the {FORCE_TARGET:.0%} target")
