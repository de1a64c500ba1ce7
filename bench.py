"""Throughput of the GPU force engine on one MI355X, in particle-steps/s.

Default workload: 50,000 bidisperse spheres (radii 1.0 / 1.4, 50:50 by number),
phi = 0.55, Pe = 10 (gammadot = 0.009, kT = 6 pi eta 0.009 / 10), mu = 0.5,
k_n = 1e4, k_t = 2/7 k_n, dt = 1e-4, xi_cut = 0.05, xi_min = 1e-3, FP64,
seeded relaxed packing, all inputs resident in HBM before timing.

Prints one JSON line.  Besides the headline FP64 number it reports the mixed
precision form on the same workload, the roofline of the pair-force kernel
(algorithmic bytes / measured kernel time against 8 TB/s) and the FP64 CPU
oracle timed on a bounded sample of the same workload on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def pair_bytes_per_particle(mixed, k, c):
    """Algorithmic HBM bytes of one pair-force launch per particle (j gathers excluded:
    Morton order serves them from cache).  k = list entries, c = live springs per particle."""
    if mixed:
        # read: pos(x,y,z,a) 32, v/w FP32 copies 24, v/w FP64 for kick 2 48, id 4, count 4, masks 8
        # write: F, T FP32 24, v, w FP64 48, masks 16; list 4k; springs FP32 read+write 24c
        return 32 + 24 + 48 + 4 + 4 + 8 + 24 + 48 + 16 + 4 * k + 24 * c
    # read: pos 32, v, w 48, id 4, count 4, masks 8; write: F, T 48, v, w 48, masks 16;
    # list 4k; springs FP64 read+write 48c
    return 32 + 48 + 4 + 4 + 8 + 48 + 48 + 16 + 4 * k + 48 * c


def eta_r(series, gd, eta, drag_xy):
    """Relative viscosity per step, Sec. II.E: (contact + lubrication + drag) xy / (eta gammadot)."""
    return (series[:, 0, 0, 1] + series[:, 1, 0, 1] + drag_xy) / (eta * gd)


def block_se(x, nb=10):
    import numpy as np
    if len(x) < nb:
        return float("nan")
    b = np.array_split(np.asarray(x), nb)
    m = np.array([t.mean() for t in b])
    return float(m.std(ddof=1) / np.sqrt(nb))


def run_gpu(P, st, precision, steps, warmup, prof_steps):
    import numpy as np
    import torch
    cfg = P.Config(box=st["L"], precision=precision, **st["params"])
    sim = P.Sim(cfg, st["radii"], st["x"], st["v"], st["w"])
    sim.step(warmup)
    sim.stress_series()
    sim.reset_stress()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ser = []
    # series ring holds 8192 steps; read what is available (latest steps)
    ser = sim.stress_series()
    stats = sim.stats()
    drag = sim.stress(0, P.STRESS_DRAG)[0, 1]
    mean = sim.stress(0, P.STRESS_TOTAL, P.STRESS_MEAN)[0, 1]
    # pair-kernel timing with HIP events on the library stream
    sim.profile(True)
    sim.step(prof_steps)
    launches, ms = sim.kernel_time()
    sim.profile(False)
    stats2 = sim.stats()
    p = st["params"]
    er = eta_r(ser, p["gammadot"], p["eta"], drag)
    sim.close()
    return dict(seconds=t1 - t0, stats=stats, stats_prof=stats2, eta_mean=mean / (p["eta"] * p["gammadot"]),
                eta_series=er, pair_ms=ms / max(launches, 1), launches=launches)


def cpu_baseline(st, seconds_target=15.0):
    from oracle import oracle as O
    o = O.Oracle(O.Params(L=st["L"], **st["params"], flags=O.CELLS), st["radii"], st["x"], st["v"], st["w"])
    n = len(st["radii"])
    t0 = time.perf_counter()
    o.step(2)
    dt2 = time.perf_counter() - t0
    k = max(2, int(seconds_target / max(dt2 / 2, 1e-6)))
    t0 = time.perf_counter()
    o.step(k)
    el = time.perf_counter() - t0
    return dict(value=n * k / el, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"{k} steps of the same {n}-particle workload after 2 warm-up steps, single thread, "
                       f"FP64, cell list rebuilt every step ({el:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--prof-steps", type=int, default=500)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3"])
    ap.add_argument("--variants", action="store_true",
                    help="only run 20 steps of each pair-kernel variant (a counter-collection driver)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the engine has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    import paper_2307_13802_amd as P
    from inputs import gen

    wl = gen.C2 if args.workload == "c2" else gen.C3
    st = gen.make_state(wl)
    n = len(st["radii"])
    print(f"workload ready: {wl.name}", file=sys.stderr, flush=True)
    if args.variants:
        for prec in (P.FP64, P.MIXED):
            for kern, lanes in ((P.KERNEL_LANES, 1), (P.KERNEL_LANES, 2), (P.KERNEL_LANES, 4),
                                (P.KERNEL_WAVE, 1), (P.KERNEL_WAVE, 2)):
                cfg = P.Config(box=st["L"], precision=prec, lanes=lanes, pair_kernel=kern, **st["params"])
                sim = P.Sim(cfg, st["radii"], st["x"], st["v"], st["w"])
                sim.step(20)
                torch.cuda.synchronize()
                sim.close()
                print(f"variant precision={prec} kernel={kern} lanes={lanes} done", file=sys.stderr, flush=True)
        return
    f64 = run_gpu(P, st, P.FP64, args.steps, args.warmup, args.prof_steps)
    print(f"fp64 done: {n * args.steps / f64['seconds']:.3e} particle-steps/s", file=sys.stderr, flush=True)
    mix = None
    if not args.no_mixed:
        mix = run_gpu(P, st, P.MIXED, args.steps, args.warmup, args.prof_steps)
        print(f"mixed done: {n * args.steps / mix['seconds']:.3e} particle-steps/s", file=sys.stderr, flush=True)

    value = n * args.steps / f64["seconds"]
    k = f64["stats_prof"]["neighbours_per_particle"]
    c = f64["stats_prof"]["contacts_per_particle"]
    bpp = pair_bytes_per_particle(False, k, c)
    achieved = bpp * n / (f64["pair_ms"] * 1e-3) / 1e9
    out = {
        "metric": "particle-steps/s + % HBM roofline; FP32-mixed vs FP64 at stated viscosity error",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["seconds"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded relaxed bidisperse packing",
        "config": {"workload": wl.name, "n": n, "phi": wl.phi, "pe": wl.pe,
                   "gammadot": st["params"]["gammadot"], "kT": st["params"]["kT"], "mu": wl.mu,
                   "dt": wl.dt, "hip_graph": True,
                   "pair_kernel": {1: "lanes", 2: "wave"}[f64["stats"]["pair_kernel"]],
                   "lanes_per_particle": f64["stats"]["lanes"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_pair<false>", "kernel_ms": f64["pair_ms"], "bytes_per_particle": bpp,
                     "list_per_particle": k, "contacts_per_particle": c},
        "eta_r_fp64": f64["eta_mean"],
    }
    if mix is not None:
        vm = n * args.steps / mix["seconds"]
        km = mix["stats_prof"]["neighbours_per_particle"]
        cm = mix["stats_prof"]["contacts_per_particle"]
        bm = pair_bytes_per_particle(True, km, cm)
        am = bm * n / (mix["pair_ms"] * 1e-3) / 1e9
        se = np.hypot(block_se(f64["eta_series"]), block_se(mix["eta_series"]))
        out["mixed"] = {"value": vm, "ms_per_step": mix["seconds"] * 1e3 / args.steps, "dtype": "f32 pair / f64 state",
                        "pair_kernel": {1: "lanes", 2: "wave"}[mix["stats"]["pair_kernel"]],
                        "lanes_per_particle": mix["stats"]["lanes"],
                        "speedup_vs_fp64": vm / value, "pair_kernel_ms": mix["pair_ms"],
                        "roofline_frac": am / HBM_PEAK_GBS, "achieved_GBs": am,
                        "eta_r": mix["eta_mean"],
                        "eta_r_rel_diff_free_running": (mix["eta_mean"] - f64["eta_mean"]) / f64["eta_mean"],
                        "eta_r_diff_std_err": float(se / abs(f64["eta_mean"]))}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(st)
        print("cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
