"""Throughput of the GPU force engine on one MI355X, in particle-steps/s.

Default workload: 50,000 bidisperse spheres (radii 1.0 / 1.4, 50:50 by number),
phi = 0.55, Pe = 10 (gammadot = 0.009, kT = 6 pi eta 0.009 / 10), mu = 0.5,
k_n = 1e4, k_t = 2/7 k_n, dt = 1e-4, xi_cut = 0.05, xi_min = 1e-3, FP64,
seeded relaxed packing, all inputs resident in HBM before timing.

Prints one JSON line.  Besides the headline FP64 number it reports the mixed
precision form on the same workload, the roofline of the pair-force kernel
(algorithmic bytes / measured kernel time against 8 TB/s, with the measured
traffic when the committed counter summary matches the kernel source) and the FP64 CPU
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


KERNEL_SRC = os.path.join(ROOT, "paper_2307_13802_amd", "csrc", "susp_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_kernel_traffic.json")
VALU_PEAK = 256 * 4 * 2.4e9  # VALU issue slots per second: 256 CUs x 4 SIMDs x 2.4 GHz


def half_bytes_per_particle(mixed, k, p, c):
    """Algorithmic HBM bytes per particle of one half-pair kernel launch (partner gathers
    excluded: Morton order serves them from cache).  k = list entries, p = interacting
    pair sides, c = contact pair sides per particle; each pair is evaluated once, so a
    particle owns p/2 pairs and c/2 contacts."""
    own = 24 + 8 + 24 + 4 if mixed else 24 + 8 + 48 + 4   # x, a, v and w (FP32 copies in mixed), id
    vec = 12 if mixed else 24                              # one 3-vector
    return (own + 4 * k / 2                                # the half of the list with higher-id partners
            + 2 * vec * c / 2                              # spring read and written per contact
            + vec * p / 2 + vec * c / 2                    # pair force; n x k_t s of a contact
            + 8 + 8 + 8 + 2)                               # interaction, contact, sliding masks; queue offset


def gather_bytes_per_particle(mixed, k, p, c):
    """Algorithmic HBM bytes per particle of one gather launch with the next step's kick
    and drift fused: own state in and out, the list, every pair record once."""
    vec = 12 if mixed else 24
    own_in = 24 + 8 + 48 + 4 + 8                           # x, a, v, w, id, displacement bound
    own_out = 24 + 48 + 8 + (24 if mixed else 0)           # x, v, w, bound (+ FP32 copies)
    return own_in + own_out + 4 * k + k + vec * p / 2 + vec * c / 2


def counter_record(lanes, n, occ):
    """The committed counter record of the half-pair kernel on the 50,000-sphere workload, if it
    was taken from the current kernel source in the same launch configuration (lanes per
    particle, form) and size as the timed run."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if (rec.get("kernel_source_sha1") != sha or rec.get("lanes") != lanes or rec.get("n") != n
            or rec.get("occupancy_form", 0) != occ):
        return None
    return rec


def measured_traffic(mixed, lanes, n, occ):
    """HBM bytes per launch of the half-pair kernel (calibrated FETCH_SIZE + WRITE_SIZE)."""
    rec = counter_record(lanes, n, occ)
    t = None if rec is None else rec.get("mixed" if mixed else "fp64", {}).get("k_half")
    return None if t is None else t["fetch_bytes"] + t["write_bytes"]


def measured_valu(mixed, lanes, n, occ):
    """VALU-busy SIMD-cycles per launch of the half-pair kernel (4 x SQ_ACTIVE_INST_VALU)."""
    rec = counter_record(lanes, n, occ)
    v = None if rec is None else rec.get("valu_busy_simd_cycles", {})
    return None if not v else v.get("mixed" if mixed else "fp64")


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
    # per-stage kernel timing with HIP events on the library stream
    sim.profile(True)
    sim.step(prof_steps)
    stage = [sim.stage_time(k) for k in range(3)]
    sim.profile(False)
    stats2 = sim.stats()
    p = st["params"]
    er = eta_r(ser, p["gammadot"], p["eta"], drag)
    sim.close()
    n_l = max(stage[1][0], 1)
    return dict(seconds=t1 - t0, stats=stats, stats_prof=stats2, eta_mean=mean / (p["eta"] * p["gammadot"]),
                eta_series=er, pair_ms=stage[1][1] / n_l, gather_ms=stage[2][1] / n_l,
                integrate_ms=stage[0][1] / n_l, launches=stage[1][0])


def roofline(r, mixed, n):
    """Roofline object of the dominant kernel (the pair kernel) from a run_gpu result."""
    st = r["stats_prof"]
    k, p, c = st["neighbours_per_particle"], st["interacting_per_particle"], st["contacts_per_particle"]
    half = st["pair_kernel"] == 3
    if half:
        bpp = half_bytes_per_particle(mixed, k, p, c)
        name = "k_half<%s>" % ("true" if mixed else "false")
    else:  # a kernel evaluating every pair from both sides, with one-body terms and kick 2
        bpp = 2 * half_bytes_per_particle(mixed, k, p, c) + 48
        name = "k_pair<%s>" % ("true" if mixed else "false")
    achieved = bpp * n / (r["pair_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(mixed, st["lanes"], n, st["occupancy_form"]) if half else None
    valu = measured_valu(mixed, st["lanes"], n, st["occupancy_form"]) if half else None
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": name, "kernel_ms": r["pair_ms"],
           "bytes_per_particle": bpp, "list_per_particle": k, "interacting_per_particle": p,
           "contacts_per_particle": c}
    if valu is not None:
        # the kernel is bound by load latency and VALU issue rather than by HBM: the VALU-busy
        # cycles (counters) per second of its time, against 256 CUs x 4 SIMDs x 2.4 GHz
        va = valu / (r["pair_ms"] * 1e-3)
        out["alu"] = {"bound": "alu", "achieved": va, "peak": VALU_PEAK, "unit": "VALU-busy SIMD-cycles/s",
                      "frac": va / VALU_PEAK}
    if half:
        gb = gather_bytes_per_particle(mixed, k, p, c)
        out["gather"] = {"kernel": "k_gather<%s>" % ("true" if mixed else "false"), "kernel_ms": r["gather_ms"],
                         "bytes_per_particle": gb,
                         "frac": gb * n / (r["gather_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


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


def eta_now(sim, P, r, gd, eta):
    """Relative viscosity of the last evaluation of replica r (contact + lubrication + drag, Sec. IV.D)."""
    return sim.stress(r, P.STRESS_TOTAL, P.STRESS_LAST)[0, 1] / (eta * gd)


def pair_time(sim, steps=100):
    """Average pair-kernel duration (ms) over `steps` steps, HIP events on the library stream."""
    sim.profile(True)
    sim.step(steps)
    launches, ms = sim.stage_time(1)
    sim.profile(False)
    return ms / max(launches, 1)


def hbm_frac(stats, mixed, n, ms):
    """Fraction of the HBM roofline of the pair kernel from its algorithmic bytes."""
    k, p, c = stats["neighbours_per_particle"], stats["interacting_per_particle"], stats["contacts_per_particle"]
    bpp = half_bytes_per_particle(mixed, k, p, c)
    if stats["pair_kernel"] != 3:
        bpp = 2 * bpp + 48
    return bpp * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS


def run_mixed_vs_fp64(P, st, steps, sample_every, say):
    """One workload in FP64 and in mixed precision from the same state and seed.

    Viscosity error, two protocols:
      * shadow: every `sample_every` steps the FP64 trajectory's state (positions,
        velocities, springs, offset, step counter) is injected into an FP64 and a
        mixed handle, which evaluate it; the relative difference of eta_r at
        identical states is recorded, and of its mean over the samples;
      * free-running: both precisions integrate independently; the difference of
        the mean eta_r over the run is compared with its block standard error.
    """
    import numpy as np
    import torch
    p = st["params"]
    gd, eta = p["gammadot"], p["eta"]
    n = len(st["radii"])
    mk = lambda prec: P.Sim(P.Config(box=st["L"], precision=prec, **p), st["radii"], st["x"], st["v"], st["w"])
    traj = mk(P.FP64)
    probe64 = mk(P.FP64)
    probe32 = mk(P.MIXED)
    say(f"  handles ready (n={n})")
    t64 = 0.0
    sh64, sh32 = [], []
    done = 0
    while done < steps:
        k = min(sample_every, steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        traj.step(k)
        torch.cuda.synchronize()
        t64 += time.perf_counter() - t0
        done += k
        s = traj.get_state()
        cij, cs, _ = traj.contacts()
        for pr, acc in ((probe64, sh64), (probe32, sh32)):
            pr.set_state(0, s["x"], s["v"], s["w"], s_le=s["s_le"], step=s["step"], contacts=(cij, cs))
            acc.append(eta_now(pr, P, 0, gd, eta))
    say(f"  fp64 trajectory + {len(sh64)} shadow samples done")
    drag = traj.stress(0, P.STRESS_DRAG)[0, 1]
    ser64 = eta_r(traj.stress_series()[-steps:], gd, eta, drag)
    st64 = traj.stats()
    ms64 = pair_time(traj)
    st64p = traj.stats()
    for h in (traj, probe64, probe32):
        h.close()
    free = mk(P.MIXED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    free.step(steps)
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    ser32 = eta_r(free.stress_series()[-steps:], gd, eta, drag)
    st32 = free.stats()
    ms32 = pair_time(free)
    st32p = free.stats()
    free.close()
    say(f"  mixed free run done")
    sh64, sh32 = np.array(sh64), np.array(sh32)
    rel = (sh32 - sh64) / np.abs(sh64)
    se = float(np.hypot(block_se(ser64), block_se(ser32)))
    m64, m32 = float(ser64.mean()), float(ser32.mean())
    k64, c64 = st64p["neighbours_per_particle"], st64p["contacts_per_particle"]
    return {
        "fp64": {"value": n * steps / t64, "pair_kernel_ms": ms64, "hbm_frac": hbm_frac(st64p, False, n, ms64),
                 "pair_kernel": {1: "lanes", 2: "wave", 3: "half"}[st64["pair_kernel"]], "lanes": st64["lanes"],
                 "occupancy_form": st64["occupancy_form"],
                 "rebuilds": st64["rebuilds"], "eta_r_mean": m64},
        "mixed": {"value": n * steps / t32, "pair_kernel_ms": ms32, "hbm_frac": hbm_frac(st32p, True, n, ms32),
                  "pair_kernel": {1: "lanes", 2: "wave", 3: "half"}[st32["pair_kernel"]], "lanes": st32["lanes"],
                  "rebuilds": st32["rebuilds"], "eta_r_mean": m32},
        "mixed_speedup": (n * steps / t32) / (n * steps / t64),
        "shadow": {"samples": int(len(rel)), "every_steps": sample_every,
                   "eta_r_rel_err_max": float(np.abs(rel).max()),
                   "eta_r_mean_rel_err": float((sh32.mean() - sh64.mean()) / abs(sh64.mean())),
                   "eta_r_fp64_mean": float(sh64.mean())},
        "free_running": {"eta_r_rel_diff": (m32 - m64) / abs(m64), "std_err_rel": se / abs(m64),
                         "within_3_se": bool(abs(m32 - m64) <= 3 * se)},
        "contacts_per_particle": c64, "sliding_fraction": st64p["sliding_fraction"],
        "list_per_particle": k64,
    }


def bench_c3(P, gen, steps, sample_every, say):
    out = {}
    for pe in (0.1, 10.0, 1000.0):
        wl = gen.Workload(f"bidisperse N=1000000 phi=0.56 Pe={pe:g}", 1_000_000, 0.56, pe, steps=steps)
        st = gen.make_state(wl)
        say(f"workload ready: {wl.name}")
        out[f"Pe={pe:g}"] = run_mixed_vs_fp64(P, st, steps, sample_every, say)
        say(f"Pe={pe:g}: fp64 {out[f'Pe={pe:g}']['fp64']['value']:.3e}  mixed {out[f'Pe={pe:g}']['mixed']['value']:.3e}")
    return out


def bench_sweep(P, gen, steps, warmup, say):
    """64 replicas of uneven N, phi, Pe and seed in one handle (mixed and FP64),
    against the same replicas stepped one handle at a time."""
    import numpy as np
    import torch
    wls = gen.sweep_replicas(64)
    sts = []
    for r, wl in enumerate(wls):
        sts.append(gen.make_state(wl))
        if r % 8 == 7:
            say(f"  packed {r + 1}/64 replicas")
    ntot = sum(len(s["radii"]) for s in sts)
    res = {"replicas": len(wls), "particles": ntot,
           "n_range": [min(w.n for w in wls), max(w.n for w in wls)]}
    for name, prec in (("mixed", P.MIXED), ("fp64", P.FP64)):
        cfgs = [P.Config(box=s["L"], precision=prec, **s["params"]) for s in sts]
        sim = P.Sim(cfgs, [s["radii"] for s in sts], [s["x"] for s in sts], [s["v"] for s in sts],
                    [s["w"] for s in sts])
        sim.step(warmup)
        sim.reset_stress()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        eta = [float(sim.stress(r, P.STRESS_TOTAL, P.STRESS_MEAN)[0, 1] / (w.eta * w.rates()[0]))
               for r, w in enumerate(wls)]
        stt = sim.stats(0)
        ms = pair_time(sim)
        sim.close()
        res[name] = {"value": ntot * steps / el, "ms_per_step": el * 1e3 / steps, "pair_kernel_ms": ms,
                     "pair_kernel": {1: "lanes", 2: "wave", 3: "half"}[stt["pair_kernel"]], "lanes": stt["lanes"],
                     "occupancy_form": stt["occupancy_form"],
                     "eta_r_mean_min": min(eta), "eta_r_mean_max": max(eta)}
        if name == "mixed":
            eta_mixed = np.array(eta)
        else:
            res["eta_r_rel_diff_max"] = float(np.max(np.abs(eta_mixed - np.array(eta)) / np.abs(np.array(eta))))
        say(f"  batched {name}: {res[name]['value']:.3e} particle-steps/s")
    # unbatched: one handle per replica, same steps, mixed
    k = max(steps // 10, 50)
    tot = 0.0
    for s in sts:
        h = P.Sim(P.Config(box=s["L"], precision=P.MIXED, **s["params"]), s["radii"], s["x"], s["v"], s["w"])
        h.step(min(warmup, 50))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.step(k)
        torch.cuda.synchronize()
        tot += time.perf_counter() - t0
        h.close()
    res["unbatched_mixed"] = {"value": ntot * k / tot, "steps_each": k}
    res["batched_speedup_vs_unbatched"] = res["mixed"]["value"] / res["unbatched_mixed"]["value"]
    res["batched_mixed_vs_fp64"] = res["mixed"]["value"] / res["fp64"]["value"]
    return res


def bench_large(P, gen, steps, warmup, say):
    """4,000,000 log-normal spheres, phi = 0.58, mu = 1, Pe = 1000, mixed precision."""
    import torch
    wl = gen.C5
    st = gen.make_state(wl)
    n = len(st["radii"])
    say(f"workload ready: {wl.name}")
    p = st["params"]
    sim = P.Sim(P.Config(box=st["L"], precision=P.MIXED, **p), st["radii"], st["x"], st["v"], st["w"])
    sim.step(warmup)
    sim.reset_stress()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(2000, steps - done)
        sim.step(k)
        done += k
        torch.cuda.synchronize()
        say(f"  {done}/{steps} steps")
    el = time.perf_counter() - t0
    stt = sim.stats()
    S = sim.stress(0, P.STRESS_TOTAL, P.STRESS_MEAN)
    ms = pair_time(sim)
    stp = sim.stats()
    sim.close()
    return {"workload": wl.name, "n": n, "value": n * steps / el, "ms_per_step": el * 1e3 / steps,
            "steps": steps, "pair_kernel_ms": ms, "hbm_frac": hbm_frac(stp, True, n, ms),
            "pair_kernel": {1: "lanes", 2: "wave", 3: "half"}[stt["pair_kernel"]], "lanes": stt["lanes"],
            "contacts_per_particle": stt["contacts_per_particle"], "sliding_fraction": stt["sliding_fraction"],
            "max_overlap": stt["max_overlap"], "rebuilds": stt["rebuilds"],
            "stress_total_mean": S.tolist(), "eta_r_mean": S[0, 1] / (p["eta"] * p["gammadot"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--prof-steps", type=int, default=500)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "sweep", "large"],
                    help="c2: 50,000 spheres (headline); c3: 1,000,000 spheres, mixed vs FP64 at three Pe; "
                         "sweep: 64 batched replicas; large: 4,000,000 log-normal spheres")
    ap.add_argument("--sample-every", type=int, default=250, help="c3: steps between shadow samples")
    ap.add_argument("--variants", action="store_true",
                    help="only run 20 steps of each pair-kernel variant (a counter-collection driver)")
    ap.add_argument("--trace", action="store_true",
                    help="profiler driver: a 256 MiB device copy (the calibration of the byte counters), then "
                         "--steps steps of the workload (c2, or c3 at Pe = 10) in FP64 and in mixed precision "
                         "with the pair kernel --pair-kernel / --lanes (a profiler distorts the timed choice)")
    ap.add_argument("--pair-kernel", type=int, default=3, help="--trace: 0 auto, 1 lanes, 2 wave, 3 half")
    ap.add_argument("--lanes", type=int, default=1, help="--trace: lanes per particle (0 = auto)")
    ap.add_argument("--form", default="auto", choices=["auto", "latency", "occupancy"],
                    help="--trace, FP64 half-pair kernel: its form (auto = chosen by timing at creation)")
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

    say = lambda m: print(m, file=sys.stderr, flush=True)
    if args.trace:
        x = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        torch.mul(x, 2.0, out=y)  # one elementwise kernel: 256 MiB read + 256 MiB written
        torch.cuda.synchronize()
        del x, y
        wl = gen.C2 if args.workload == "c2" else gen.C3
        st = gen.make_state(wl)
        say(f"workload ready: {wl.name}")
        form = {"auto": 0, "latency": P.HALF_OCC_OFF, "occupancy": P.HALF_OCC_ON}[args.form]
        for prec in (P.FP64, P.MIXED):
            sim = P.Sim(P.Config(box=st["L"], precision=prec, pair_kernel=args.pair_kernel, lanes=args.lanes,
                                 flags=form if prec == P.FP64 else 0, **st["params"]),
                        st["radii"], st["x"], st["v"], st["w"])
            stt = sim.stats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(args.steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            sim.close()
            say(f"precision={prec} kernel={stt['pair_kernel']} lanes={stt['lanes']} "
                f"occupancy_form={stt['occupancy_form']}: {args.steps} steps, "
                f"{len(st['radii']) * args.steps / el:.3e} particle-steps/s")
        return
    if args.workload in ("c3", "sweep", "large"):
        steps = args.steps if args.steps != 10000 or args.workload == "large" else 5000
        if args.workload == "c3":
            res = {"workload": "bidisperse N=1000000 phi=0.56, Pe in {0.1, 10, 1000}, mixed vs FP64",
                   "steps": steps, "results": bench_c3(P, gen, steps, args.sample_every, say)}
        elif args.workload == "sweep":
            res = {"workload": "64 replicas, N in [2000, 20000], phi in {0.45, 0.50, 0.54, 0.58}, "
                               "Pe log-spaced 1e-2..1e3, seeds 0..63",
                   "steps": steps, "results": bench_sweep(P, gen, steps, args.warmup, say)}
        else:
            res = bench_large(P, gen, args.steps, args.warmup, say)
        res["unit"] = "particle-steps/s"
        print(json.dumps(res), flush=True)
        return
    wl = gen.C2
    st = gen.make_state(wl)
    n = len(st["radii"])
    print(f"workload ready: {wl.name}", file=sys.stderr, flush=True)
    if args.variants:
        for prec in (P.FP64, P.MIXED):
            for kern, lanes in ((P.KERNEL_LANES, 1), (P.KERNEL_LANES, 2), (P.KERNEL_LANES, 4),
                                (P.KERNEL_WAVE, 1), (P.KERNEL_WAVE, 2), (P.KERNEL_HALF, 1)):
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
                   "pair_kernel": {1: "lanes", 2: "wave", 3: "half"}[f64["stats"]["pair_kernel"]],
                   "lanes_per_particle": f64["stats"]["lanes"],
                   "occupancy_form": f64["stats"]["occupancy_form"]},
        "roofline": roofline(f64, False, n),
        "eta_r_fp64": f64["eta_mean"],
    }
    if mix is not None:
        vm = n * args.steps / mix["seconds"]
        rm = roofline(mix, True, n)
        se = np.hypot(block_se(f64["eta_series"]), block_se(mix["eta_series"]))
        out["mixed"] = {"value": vm, "ms_per_step": mix["seconds"] * 1e3 / args.steps, "dtype": "f32 pair / f64 state",
                        "pair_kernel": {1: "lanes", 2: "wave", 3: "half"}[mix["stats"]["pair_kernel"]],
                        "lanes_per_particle": mix["stats"]["lanes"],
                        "occupancy_form": mix["stats"]["occupancy_form"],
                        "speedup_vs_fp64": vm / value, "roofline": rm,
                        "eta_r": mix["eta_mean"],
                        "eta_r_rel_diff_free_running": (mix["eta_mean"] - f64["eta_mean"]) / f64["eta_mean"],
                        "eta_r_diff_std_err": float(se / abs(f64["eta_mean"]))}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(st)
        print("cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
