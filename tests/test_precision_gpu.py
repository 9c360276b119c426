"""Storage precision: FP32, shifted FP16 and shifted BF16 population storage against the
FP64 oracle on the two-capsule film box (128 x 128 x 64, two anchored capsules R = 10,
ks = 0.05) after 1000 and 5000 steps, and on the precision-form box (256 x 256 x 96, the
same film and plane, 16 anchored capsules R = 10 at seeded random positions, ks = 0.05)
after 1000, 5000 and 10000 steps.

The reference values are the oracle's, written by tests/golden/make_precision_reference.py.
Measured quantities: meniscus height h(x, y) over the columns where both sides define it
(max and RMS of |dh|, in lattice units), the capillary force on each capsule (relative
error of the vector), and the mass drift of each component relative to its initial mass.

On the two-capsule box FP32 storage is held to the bounds of the FP32 parity tests.  The
16-capsule box is more sensitive: its contact lines move in discrete jumps, and the step at
which one jumps is decided by rounding, so after 1000 steps FP32 arithmetic alone moves the
capillary force of a capsule by up to a quarter (the oracle's own FP32 build against its
FP64 build, ``c3_precision_oracle_f32.npz``); there FP32 storage has to stay within that
envelope.  The 16-bit errors have no closed form (parity unpinned): they are measured and
printed, held to about 1.5 times the value measured (2 times at 10000 steps on the
16-capsule box, where every storage has left the reference trajectory), and a storage that
misses the 1 % capillary-force target is reported as an expected failure (xfail) after
those bounds pass.  Each constant-shift 16-bit format runs
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

# (storage, rho_shift, bounds per workload and checkpoint: max |dh|, rms |dh|, relative
# capillary force error, mass drift).  The runs are bitwise deterministic; each 16-bit bound
# is the value measured with the present kernels times about 1.5 (2 at 10000 steps), so a
# codec change that loses precision fails here.
FP32_BOUNDS = (1e-2, 1e-3, 1e-2, 1e-5)
CASES = [
    ("f32", (1.0, 1.0), {"c2": {5000: FP32_BOUNDS},
                         "c3": {1000: (1.2e-2, 9e-5, 8e-2, 5.3e-7),
                                10000: (0.89, 5.1e-2, 1.7, 1.1e-5)}}),
    ("f16", (1.0, 1.0), {"c2": {5000: (1.8, 0.7, 1.8, 3.5e-2)},
                         "c3": {1000: (0.94, 0.26, 4.9, 1.1e-3), 10000: (6.1, 2.0, 29.0, 4.5e-3)}}),
    ("f16", (0.0, 0.0), {"c2": {5000: (1.1, 0.4, 0.6, 4e-3)},
                         "c3": {1000: (0.41, 0.2, 2.5, 1.9e-3), 10000: (2.4, 0.76, 7.7, 3.2e-3)}}),
    ("bf16", (1.0, 1.0), {"c2": {5000: (4.0, 0.9, 7.0, 1.5e-2)},
                          "c3": {1000: (1.9, 0.39, 25.5, 6.4e-3), 10000: (8.0, 2.1, 17.0, 8.3e-3)}}),
    ("bf16", (0.0, 0.0), {"c2": {5000: (3.2, 0.85, 1.4, 1.1e-2)},
                          "c3": {1000: (1.6, 0.44, 7.2, 1.8e-2), 10000: (6.7, 2.0, 13.7, 1.03e-2)}}),
    ("f16site", (0.0, 0.0), {"c2": {5000: (0.31, 0.05, 0.85, 8.6e-5)},
                             "c3": {1000: (3.7e-2, 7.7e-4, 0.48, 1.7e-5),
                                    10000: (0.77, 4.6e-2, 4.0, 1.6e-4)}}),
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
    for cp, (hmax, hrms, fcap, drift) in bounds[workload].items():
        r = res[cp]
        assert r["dh_max"] <= hmax and r["dh_rms"] <= hrms, (cp, r)
        assert r["fcap"] <= fcap, (cp, r)
        assert r["drift"] <= drift, (cp, r)
    env_path = os.path.join(GOLDEN, f"{workload}_precision_oracle_f32.npz")
    if storage == "f32" and os.path.exists(env_path):
        # the deviation of the oracle's own FP32 build from its FP64 build bounds what FP32
        # arithmetic alone does to these quantities; FP32 storage has to stay inside it
        env = np.load(env_path, allow_pickle=False)
        for cp in [int(c) for c in env["checkpoints"]]:
            e = errors(ref, cp, env[f"meniscus_{cp}"].astype(np.float64),
                       [dict(f_capillary=f, f_anchor=a) for f, a in
                        zip(env[f"f_capillary_{cp}"], env[f"f_anchor_{cp}"])],
                       env[f"mass_{cp}"])
            r = res[cp]
            print(f"  step {cp}: oracle FP32 build against FP64: max|dh| {e['dh_max']:.3e}, "
                  f"rms|dh| {e['dh_rms']:.3e}, capillary force {e['fcap']:.3e}, mass drift "
                  f"{e['drift']:.2e}", flush=True)
            assert r["dh_max"] <= e["dh_max"] and r["dh_rms"] <= e["dh_rms"]
            assert r["fcap"] <= e["fcap"] and r["fanc"] <= e["fanc"]
    r = res[max(res)]
    if storage != "f32" and r["fcap"] > FORCE_TARGET:
        pytest.xfail(f"{storage} shift {shift}: capillary force error {r['fcap']:.2e} above "
                     f"the {FORCE_TARGET:.0%} target")
