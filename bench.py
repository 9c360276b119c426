"""Throughput of the fused two-component D3Q19 + capsule time step on one MI355X.

Workload: the 256 x 256 x 96 film-drying box with 16 capsules R = 10 (5120 triangles
each, seeded random positions), wall at z = 0, film 12 layers high, repulsive plane 10
lattice units above the wall.  A step is one pass of the whole hot path (labels,
membrane forces, spreading, fused fluid step, interpolation/advection).

Prints one JSON line: MLUPS (fluid-site updates per microsecond, both components count
as one update) for FP32 population storage, the HBM roofline of the dominant kernel
(the fluid step) measured with HIP events on the library's stream, the same figures for
the FP16 / BF16 storage shifted by a constant and the FP16 storage shifted by each site's
own density (FP32 density per site beside it), the batched form (64 independent capsule-pair boxes of
sizes 80x60x40 .. 128x96x48, stacked by size into slabs, one fluid launch per step over
all of them; FP32 and FP16 storage), and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the fused fluid kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE,
# scaled by the same counters on a plain 1 GiB copy (profiles/fluid_c3_f32_hbm_traffic.md),
# keyed by (storage, tile, zchunk, first-chunk offset).  Reported only for the launch shape
# it was taken on.
MEASURED_TRAFFIC_BYTES = {("f32", 11, 48, 2): 2.0277e9}
WORKLOAD = "film 256x256x96, wall, 16 capsules R=10 (5120 tri), ks=0.05"


TILES = {1: "32x8", 2: "64x4", 3: "32x16", 4: "64x8", 5: "16x16", 6: "pipe32x8",
         7: "pipe64x4", 8: "pipe16x16", 9: "pipe32x16", 10: "pipe64x8", 11: "rows256x2",
         12: "rows128x4", 13: "rows-nx"}


def tune(sim, steps=10):
    """The library's launch-shape autotuner (``lbm_autotune``): every tile shape that
    applies to this box and a few z-chunk depths, timed with HIP events, the fastest kept."""
    t = sim.autotune(steps)
    print(f"#   autotuner: tile {TILES[t['tile']]} zchunk {t['zchunk']} first chunk "
          f"{t['zoff']} planes shorter: fluid {t['fluid_ms'] * 1e3:.1f} us", file=sys.stderr,
          flush=True)
    return dict(tile=TILES[t["tile"]], tile_id=t["tile"], zchunk=t["zchunk"], zoff=t["zoff"],
                fluid_ms=t["fluid_ms"])


def run_gpu(cfg, storage, steps, warmup, do_tune=True, launch=None):
    import torch

    from paper_2007_15405_amd import Sim

    sim = Sim(cfg, storage=storage, stream="torch")
    stream = torch.cuda.current_stream()
    sim.step(2)                   # capsule windows in place before the launch shapes are timed
    tuned = tune(sim) if do_tune else None
    if launch is not None:
        sim.set_launch(launch[0], launch[1])
        zoff = launch[2] if len(launch) > 2 else 0
        sim.set_zoffset(zoff)
        tuned = dict(tile=TILES.get(launch[0], "two-kernel"), tile_id=launch[0], zchunk=launch[1],
                     zoff=zoff)
    sim.step(warmup)
    sim.sync()
    sim.kernel_stats()            # discard
    # timed region: HIP events around the fluid kernel only (two per step), so the step
    # time is not inflated by events between the other kernels
    sim.set_profiling(2)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    sim.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    sim.sync()
    ms = t0.elapsed_time(t1)
    stats = sim.kernel_stats()
    # per-kernel breakdown from a separate, untimed pass with every kernel bracketed
    sim.set_profiling(1)
    sim.step(min(steps, 50))
    breakdown = sim.kernel_stats()
    sim.set_profiling(0)
    sites = sim.fluid_sites
    bps = sim.bytes_per_site
    fl_launches, fl_ms = stats["fluid"]
    fl_avg = fl_ms / fl_launches
    achieved = bps * sites / (fl_avg * 1e-3) / 1e9
    out = dict(
        mlups=sites * steps / (ms * 1e-3) / 1e6,
        ms_per_step=ms / steps,
        fluid_ms=fl_avg,
        bytes_per_site=bps,
        fluid_sites=sites,
        achieved_gbs=achieved,
        frac=achieved / PEAK_HBM_GBS,
        kernels={k: round(v[1] / max(v[0], 1), 5) for k, v in breakdown.items()},
        launch=tuned,
    )
    sim.close()
    return out


def run_batch(storage, steps, warmup, do_tune=True, launch=None, parts=None):
    """The batched form: every group of equal box size is one handle of stacked slabs,
    and one Batch advances all groups with one fluid launch per step."""
    import torch

    import synth
    from paper_2007_15405_amd import Batch, Sim

    inst = synth.batch_instances()
    groups = synth.batch_groups(inst)
    sims = [Sim(g, storage=storage, stream="torch", meshes=synth.capsule_meshes(g["capsules"]))
            for g in groups]
    bt = Batch(sims)
    stream = torch.cuda.current_stream()
    bt.step(2)
    if launch is not None:
        bt.set_launch(*launch)
        best = (None, launch[0], launch[1])
    elif do_tune:
        t = bt.autotune(10)
        print(f"#   batch {storage} autotuner: tile {TILES[t['tile']]} zchunk {t['zchunk']}: "
              f"fluid {t['fluid_ms'] * 1e3:.1f} us", file=sys.stderr, flush=True)
        best = (t["fluid_ms"], t["tile"], t["zchunk"])
    else:
        best = (None, 10, 0)
        bt.set_launch(10, 0)

    def timed_steps():
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        bt.step(steps)
        t1.record(stream)
        torch.cuda.synchronize()
        bt.sync()
        return t0.elapsed_time(t1)

    # one part: the fluid kernel's duration (HIP events around it) for the roofline
    bt.step(warmup)
    bt.sync()
    bt.kernel_stats()
    bt.set_profiling(2)
    ms1 = timed_steps()
    n, fms = bt.kernel_stats()["fluid"]
    bt.set_profiling(1)
    bt.step(min(steps, 20))
    breakdown = bt.kernel_stats()
    bt.set_profiling(0)
    # more parts overlap one part's capsule kernels with another's fluid kernel: the
    # throughput is taken from the fastest split (no events inside the timed steps)
    per_parts = {1: ms1}
    for p in ((2, 3, 4) if parts is None else (parts,) if parts > 1 else ()):
        bt.set_parts(p)
        bt.step(warmup)
        per_parts[p] = timed_steps()
    best_parts = min(per_parts, key=per_parts.get)
    ms = per_parts[best_parts]
    # the same split replayed from captured graphs (two steps per graph launch); kept for
    # the figure if it is faster
    bt.set_parts(best_parts)
    bt.set_graph(True)
    bt.step(warmup + warmup % 2)
    ms_graph = timed_steps()
    bt.set_graph(False)
    graph = ms_graph < ms
    ms = min(ms, ms_graph)
    # the fluid launch as a resident grid taking tiles from a device work queue: its kernel
    # time with one part (as fluid_ms), then the step time with the fastest split
    bt.set_schedule(True)
    bt.set_parts(1)
    bt.step(warmup)
    bt.sync()
    bt.kernel_stats()
    bt.set_profiling(2)
    bt.step(min(steps, 20))
    nq, fq = bt.kernel_stats()["fluid"]
    bt.set_profiling(0)
    bt.set_parts(best_parts)
    bt.step(warmup)
    ms_queue = timed_steps()
    bt.set_schedule(False)
    schedule = "queue" if ms_queue < ms else "static"
    ms = min(ms, ms_queue)
    sites, bps = bt.fluid_sites, bt.bytes_per_site
    fl_avg = fms / n
    achieved = bps * sites / (fl_avg * 1e-3) / 1e9
    out = dict(
        workload=f"{len(inst)} capsule-pair boxes {min(g['nx'] for g in groups)}x"
                 f"{min(g['ny'] for g in groups)}x40 .. 128x96x48, R=10 (5120 tri), ks "
                 f"log-uniform 0.002..0.2, stacked into {len(groups)} groups of equal size",
        instances=len(inst), groups=len(groups), capsules=sum(len(g["capsules"]) for g in groups),
        fluid_sites=sites, storage=storage,
        mlups=round(sites * steps / (ms * 1e-3) / 1e6, 2), ms_per_step=round(ms / steps, 5),
        parts=best_parts,
        ms_per_step_by_parts={k: round(v / steps, 5) for k, v in per_parts.items()},
        ms_per_step_graph=round(ms_graph / steps, 5), graph=graph,
        ms_per_step_queue=round(ms_queue / steps, 5), fluid_ms_queue=round(fq / nq, 5),
        schedule=schedule,
        fluid_ms=round(fl_avg, 5), bytes_per_site=bps, achieved_gbs=round(achieved, 1),
        frac=round(achieved / PEAK_HBM_GBS, 4),
        launch=dict(tile=TILES[best[1]], tile_id=best[1], zchunk=best[2]),
        kernels_ms={k: round(v[1] / max(v[0], 1), 5) for k, v in breakdown.items()},
    )
    bt.close()
    for x in sims:
        x.close()
    return out


PEAK_BF16_TFLOPS = 2500.0


WET_MAX = 0.08     # capsule wetting offsets sampled in [-0.08, 0.08]: contact angles ~60..120 deg


def run_surrogate(seeds=tuple(range(201, 209)), steps=20000, average=10000, train_steps=500):
    """The learned form: training data from the batched solver (64 capsule-pair runs per
    seed), the network trained on three quarters of the pairs that stay out of contact,
    held-out error, training and inference speed, and the solver's time per pair."""
    import numpy as np

    import synth
    from paper_2007_15405_amd import surrogate as S
    t0 = time.perf_counter()
    parts = []
    for sd in seeds:
        parts.append(S.run_pairs(synth.batch_instances(seed=sd, wet_max=WET_MAX), steps,
                                 average=average))
        print(f"# surrogate data: seed {sd} done, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    t_lbm = time.perf_counter() - t0
    X = np.concatenate([p[0] for p in parts])
    Y = np.concatenate([p[1] for p in parts])
    keep = S.in_domain(X)
    X, Y = X[keep], Y[keep]
    idx = np.random.default_rng(1).permutation(len(X))
    te, tr = idx[: len(X) // 4], idx[len(X) // 4:]
    t1 = time.perf_counter()
    f = S.fit(X[tr], Y[tr], steps=train_steps)
    t_fit = time.perf_counter() - t1
    P = f.predict(X[te])
    err = np.linalg.norm(P - Y[te], axis=0) / np.linalg.norm(Y[te] - Y[tr].mean(0), axis=0)
    # training speed: more Adam steps on the same data (full batch)
    reps = 2000
    t2 = time.perf_counter()
    f.net.train(reps, 1e-4)
    us_step = (time.perf_counter() - t2) / reps * 1e6
    n = len(tr)
    flops = 3 * 2 * n * (4 * 64 + 64 * 64 * 2 + 64 * 2)   # forward, input and weight gradients
    # inference: 4096 queries in one call
    Q = X[np.random.default_rng(2).integers(0, len(X), 4096)]
    t3 = time.perf_counter()
    f.predict(Q)
    us_query = (time.perf_counter() - t3) / len(Q) * 1e6
    cl = run_cluster(f, X[tr], Y[tr])
    f.net.close()
    return dict(cluster_evolution=cl,
        wetting_offsets=[-WET_MAX, WET_MAX],
        contact_angle_range=[round(float(X[:, 3].min()), 2), round(float(X[:, 3].max()), 2)],
        samples=int(len(X)), train=int(len(tr)), held_out=int(len(te)),
        solver_runs=len(seeds) * 64, solver_steps=steps, outputs_averaged_over=average,
        held_out_rel_error={"lateral_force": round(float(err[0]), 4),
                            "meniscus_deformation": round(float(err[1]), 4)},
        train_steps=train_steps, fit_s=round(t_fit, 3), us_per_adam_step=round(us_step, 2),
        gemm_tflops=round(flops / (us_step * 1e-6) / 1e12, 5),
        gemm_frac_of_bf16_peak=round(flops / (us_step * 1e-6) / 1e12 / PEAK_BF16_TFLOPS, 8),
        us_per_query=round(us_query, 4), solver_s_per_pair=round(t_lbm / (len(seeds) * 64), 4),
        speedup_per_pair=round(t_lbm / (len(seeds) * 64) / (us_query * 1e-6), 1))


def run_network_kernels(samples=480, adam_steps=500, capsules=512, cluster_steps=2000):
    """The network's kernels alone on synthetic data, sized like the learned form's use:
    full-batch Adam on ``samples`` random normalised samples (initial parameters of
    ``synth.surrogate_init``), then the cluster evolution of ``capsules`` capsules at 25 %
    area fraction with normalisation of unit scale.  Wall time per Adam step and per
    cluster step."""
    import numpy as np

    import synth
    from paper_2007_15405_amd import Surrogate
    rng = np.random.default_rng(synth.SEED)
    net = Surrogate(synth.surrogate_init(), samples)
    x = rng.normal(size=(samples, 4)).astype(np.float32)
    t = np.tanh(x[:, :2] - 0.5 * x[:, 2:]).astype(np.float32)
    net.set_data(x, t)
    net.train(5, 1e-3)
    t0 = time.perf_counter()
    net.train(adam_steps, 1e-3)
    us_adam = (time.perf_counter() - t0) / adam_steps * 1e6
    box, p = synth.cluster_film(n=capsules, packing=0.25)
    cp = dict(box=box, radius=10.0, features=[-1.0, 0.2, 90.0], in_mean=[4.0, -1.0, 0.2, 90.0],
              in_scale=[1.0, 1.0, 1.0, 1.0], out_mean=[0.0, 0.0], out_scale=[1e-3, 1.0],
              r_contact=2.4, r_cut=6.0, k_contact=1e-3, mobility=50.0)
    net.cluster(p, 10, **cp)
    t0 = time.perf_counter()
    net.cluster(p, cluster_steps, **cp)
    us_cl = (time.perf_counter() - t0) / cluster_steps * 1e6
    net.close()
    pairs = capsules * (capsules - 1)
    flop = 2 * (4 * 64 + 64 * 64 * 2 + 64 * 2) * pairs
    return dict(adam_samples=samples, adam_steps=adam_steps, us_per_adam_step=round(us_adam, 2),
                cluster_capsules=capsules, cluster_steps=cluster_steps,
                us_per_cluster_step=round(us_cl, 2),
                cluster_network_tflops=round(flop / (us_cl * 1e-6) / 1e12, 3),
                cpu_baseline=network_cpu_baseline(x, t, p, cp))


def network_cpu_baseline(x, t, p, cp, reps=3):
    """The network's CPU reference (the oracle, numpy, mixed precision as the kernels)
    timed on the same data: one Adam step (loss, gradient and update) over the samples,
    and one cluster step of all capsules; best of ``reps``."""
    import numpy as np

    import synth
    from oracle import cluster, mlp
    th = synth.surrogate_init().astype(np.float64)
    z = np.zeros_like(th)
    best_adam = best_cl = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        _, g = mlp.loss_and_grad(th, x, t, mixed=True)
        mlp.adam(th, g, z, z, 1, 1e-3)
        best_adam = min(best_adam, time.perf_counter() - t0)
        t0 = time.perf_counter()
        cluster.step(th, p, cp)
        best_cl = min(best_cl, time.perf_counter() - t0)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return dict(kind="oracle", unit="us", us_per_adam_step=round(best_adam * 1e6, 1),
                us_per_cluster_step=round(best_cl * 1e6, 1), cores=threads,
                sample=f"best of {reps}: one Adam step on {len(x)} samples, one cluster step of "
                       f"{len(p)} capsules (numpy, float64 with bfloat16 operands)")


def run_cluster(f, X, Y, n=512, packing=0.25, steps=20000, every=2000, timed=2000):
    """Cluster evolution of ``n`` capsules at area fraction ``packing`` driven by the
    trained network (shear modulus and film height: the medians of the training inputs;
    mobility such that the strongest training force F moves a capsule 0.5 lattice units
    per step, contact stiffness 5 F per radius of overlap, so that an overlap shrinks by
    half per step without overshoot): time per step (one fused kernel evaluating the network for all n (n - 1)
    ordered pairs), the network's matrix-core rate, the learned force against the
    separation, and the cluster statistics of runs at the median and at the extreme
    contact angles of the training data."""
    import numpy as np

    import synth
    from paper_2007_15405_amd import surrogate as S
    box, p0 = synth.cluster_film(n=n, packing=packing)
    med = np.median(X[:, 1:], axis=0)
    fmax = float(np.abs(Y[:, 0]).max())
    mob, kc = 0.5 / fmax, 5.0 * fmax
    cp = S.cluster_params(f, med, box, k_contact=kc, mobility=mob)
    f.net.cluster(p0, 10, **cp)                               # warm-up
    t = time.perf_counter()
    f.net.cluster(p0, timed, **cp)
    us = (time.perf_counter() - t) / timed * 1e6
    pairs = n * (n - 1)
    flop = 2 * (4 * 64 + 64 * 64 * 2 + 64 * 2) * pairs
    rs = np.round(np.arange(S.CONTACT, cp["r_cut"] + 1e-9, 0.4), 2)
    runs = {}
    for ang in (X[:, 3].min(), med[2], X[:, 3].max()):
        fe = np.array([med[0], med[1], ang])
        force = f.predict(np.column_stack([rs, np.tile(fe, (len(rs), 1))]))[:, 0]
        p, hist = S.evolve(f, p0, steps, every, fe, box, k_contact=kc, mobility=mob)
        rk, g = S.rdf(p, box, 1.0, 6 * S.RADIUS)
        runs[f"{ang:.1f}"] = dict(
            learned_force_vs_L_over_R=[(float(r), float(v)) for r, v in zip(rs, np.round(force, 6))],
            mean_and_largest_cluster=[(a, round(b, 3), c) for a, b, c in hist],
            rdf_first_peak_over_2R=round(float(rk[np.argmax(g)]) / (2 * S.RADIUS), 3))
    return dict(capsules=n, area_fraction=packing, box=round(box, 2), r_cut_radii=round(cp["r_cut"], 3),
                us_per_step=round(us, 2), pair_evals_per_s=round(pairs / (us * 1e-6), 1),
                network_tflops=round(flop / (us * 1e-6) / 1e12, 3),
                frac_of_bf16_peak=round(flop / (us * 1e-6) / 1e12 / PEAK_BF16_TFLOPS, 5),
                log10_ks_and_film=[round(float(v), 4) for v in med[:2]], mobility=round(mob, 3),
                k_contact=round(kc, 4),
                steps=steps, by_contact_angle=runs)


def cpu_model() -> str:
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, steps=30, single_steps=3):
    """The FP64 oracle on the same workload on the host cores: ``steps`` steps with all
    threads (the reported value), then ``single_steps`` steps on one thread."""
    import oracle
    import synth
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    sites = synth.fluid_sites(cfg)

    def rate(threads, n):
        o = oracle.Oracle(cfg, "f64", n_threads=threads)
        o.step(1)
        t = time.perf_counter()
        o.step(n)
        dt = time.perf_counter() - t
        o.close()
        return sites * n / dt / 1e6, dt

    v, dt = rate(cores, steps)
    v1, dt1 = rate(1, single_steps)
    return dict(value=v, unit="MLUPS", cores=cores, kind="oracle", cpu_model=cpu_model(),
                sample=f"{steps} steps of the same workload after 1 warm-up step, FP64 oracle, "
                       f"{dt:.1f} s",
                single_thread=dict(value=round(v1, 3), steps=single_steps, seconds=round(dt1, 1)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="all", choices=["all", "f32", "f16", "bf16", "f16site"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched form")
    ap.add_argument("--no-bounce-back", action="store_true",
                    help="skip the bounce-back coupling leg")
    ap.add_argument("--batch-only", action="store_true", help="only the batched form")
    ap.add_argument("--network-kernels", action="store_true",
                    help="only the network's kernels on synthetic data (for kernel traces): "
                         "500 Adam steps on 480 samples, 2000 steps of the 512-capsule cluster "
                         "evolution")
    ap.add_argument("--surrogate", action="store_true",
                    help="only the learned form: solver data, training, held-out error, speed")
    ap.add_argument("--kb", type=float, default=0.0,
                    help="bending modulus of the film box's capsules (the workload has none)")
    ap.add_argument("--parts", type=int, default=None,
                    help="batched form: only this split over streams (default: try 1..4)")
    ap.add_argument("--tile", type=int, default=None, help="fixed launch shape (skips tuning)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes (counter calibration)")
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--zoff", type=int, default=0,
                    help="with --tile: planes the first z-chunk is shortened by")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); "
              f"the multi-GPU halo exchange is designed but not implemented",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calib:
        # plain copy kernel of known size: rocprofv3's FETCH_SIZE / WRITE_SIZE of this run
        # give the counter scale (bytes counted per byte moved) used for the traffic figure
        # the same copies timed with HIP events give the device's practical read + write rate
        import torch
        n = args.copy_calib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(5):
            dst.copy_(src)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / 5
        print(json.dumps(dict(copy_bytes_each_way=n * 4, launches=6, ms_per_copy=round(ms, 4),
                              read_plus_write_gbs=round(2 * n * 4 / (ms * 1e-3) / 1e9, 1))),
              flush=True)
        return

    if args.surrogate:
        print(json.dumps(dict(surrogate=run_surrogate())), flush=True)
        return
    if args.network_kernels:
        print(json.dumps(dict(network_kernels=run_network_kernels())), flush=True)
        return

    import synth
    cfg = synth.workload("c3")
    if args.kb:
        cfg["capsules"] = [dict(c, kb=args.kb) for c in cfg["capsules"]]
    res = {}
    batched = {}
    if not args.no_batch:
        for st in (["f32", "f16"] if args.storage == "all" else [args.storage]):
            batched[st] = run_batch(st, min(args.steps, 100), min(args.warmup, 10),
                                    not args.no_tune,
                                    (args.tile, args.zchunk) if args.tile is not None else None,
                                    args.parts)
            b = batched[st]
            print(f"# batch {st}: {b['mlups']:.1f} MLUPS, {b['ms_per_step']:.4f} ms/step, fluid "
                  f"{b['fluid_ms']:.4f} ms = {b['achieved_gbs']:.0f} GB/s", file=sys.stderr,
                  flush=True)
    if args.batch_only:
        print(json.dumps(dict(batched=batched)), flush=True)
        return
    for st in (["f32", "f16", "bf16", "f16site"] if args.storage == "all" else [args.storage]):
        fixed = (args.tile, args.zchunk, args.zoff) if args.tile is not None else None
        res[st] = run_gpu(cfg, st, args.steps, args.warmup, not args.no_tune and fixed is None, fixed)
        print(f"# {st}: {res[st]['mlups']:.1f} MLUPS, {res[st]['ms_per_step']:.4f} ms/step, "
              f"fluid {res[st]['fluid_ms']:.4f} ms = {res[st]['achieved_gbs']:.0f} GB/s",
              file=sys.stderr, flush=True)
    # the paper's own coupling (half-way bounce-back on the membrane, momentum exchange,
    # Newtonian nodes) on the same box, FP32 storage
    coupling = {}
    if not args.no_bounce_back:
        bcfg = dict(cfg, coupling=1)
        fixed = (args.tile, args.zchunk, args.zoff) if args.tile is not None else None
        coupling["bounce_back"] = run_gpu(bcfg, "f32", min(args.steps, 100), args.warmup,
                                          not args.no_tune and fixed is None, fixed)
        b = coupling["bounce_back"]
        print(f"# bounce-back f32: {b['mlups']:.1f} MLUPS, {b['ms_per_step']:.4f} ms/step",
              file=sys.stderr, flush=True)
    head = res["f32"] if "f32" in res else next(iter(res.values()))
    head_st = "f32" if "f32" in res else next(iter(res))
    line = dict(
        metric="MLUPS (2-comp D3Q19 + IBM capsules), % HBM roofline of the fused fluid kernel",
        value=round(head["mlups"], 2),
        unit="MLUPS",
        n_gpus=1,
        steps=args.steps,
        warmup=args.warmup,
        ms_per_step=round(head["ms_per_step"], 5),
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype="f32",
        data="synthetic",
        config=dict(workload=WORKLOAD + (f", bending kb={args.kb}" if args.kb else ""),
                    nx=256, ny=256, nz=96, capsules=16,
                    storage=head_st, fluid_sites=head["fluid_sites"]),
        roofline=dict(bound="hbm", achieved=round(head["achieved_gbs"], 1), peak=PEAK_HBM_GBS,
                      unit="GB/s", frac=round(head["frac"], 4),
                      traffic=MEASURED_TRAFFIC_BYTES.get(
                          (head_st, head["launch"]["tile_id"], head["launch"]["zchunk"],
                           head["launch"].get("zoff", 0)) if head.get("launch") else None),
                      traffic_unit="bytes per launch",
                      algorithmic_bytes=head["bytes_per_site"] * head["fluid_sites"],
                      bytes_per_site=head["bytes_per_site"], kernel="fluid",
                      kernel_ms=round(head["fluid_ms"], 5), launch=head["launch"]),
        kernels_ms=head["kernels"],
        storage_variants={k: dict(mlups=round(v["mlups"], 2), ms_per_step=round(v["ms_per_step"], 5),
                                  fluid_ms=round(v["fluid_ms"], 5),
                                  achieved_gbs=round(v["achieved_gbs"], 1),
                                  frac=round(v["frac"], 4), bytes_per_site=v["bytes_per_site"],
                                  launch=v["launch"])
                          for k, v in res.items()},
        batched=batched or None,
        couplings={k: dict(mlups=round(v["mlups"], 2), ms_per_step=round(v["ms_per_step"], 5),
                           fluid_ms=round(v["fluid_ms"], 5), kernels_ms=v["kernels"],
                           launch=v["launch"])
                   for k, v in coupling.items()} or None,
    )
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
