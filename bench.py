"""Throughput of the GPU force engine on one MI355X, in particle-steps/s.

Default workload (the metric's configuration): 1,000,000 bidisperse spheres
(radii 1.0 / 1.4, 50:50 by number), phi = 0.56, Pe = 10 (gammadot = 0.009,
kT = 6 pi eta 0.009 / 10), mu = 0.5, k_n = 1e4, k_t = 2/7 k_n, dt = 1e-4,
xi_cut = 0.05, xi_min = 1e-3, FP64, seeded relaxed packing, all inputs resident
in HBM before timing, launch and list parameters from the tuner (read from the
cache of parameters it measured on an MI355X, so that reruns time the same launch).

Prints one JSON line: the FP64 throughput (headline), the mixed-precision form on
the same workload with its viscosity error under the shadow protocol (FP64 states
evaluated in both precisions), the roofline of the pair-force kernel (algorithmic
bytes of the hot-path scope table / measured kernel time, against 8 TB/s; the
measured HBM traffic when a committed counter summary matches the kernel source
and launch configuration) and the FP64 CPU oracle timed on a bounded prefix of
the same workload on the host.
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
# counter summary of the pair kernel on the default workload (HBM traffic, VALU busy fraction)
COUNTER_FILE = os.path.join(ROOT, "profiles", "counters_pair_kernel_bidisperse_N1000000_phi0.56.txt")


def pair_bytes_per_particle(mixed, k, c):
    """Algorithmic HBM bytes per particle of one pair-force launch, as the hot-path scope
    table counts them: own state (x, a, v, w, id: 84 B FP64, 56 B mixed), the list (4 B per
    entry, k entries), the contact history read and written (52 B per contact FP64, 28 B
    mixed; c contacts per particle) and F, T written (48 B / 24 B).  Partner gathers are
    not counted (the cell order serves them from cache)."""
    return (56 + 4 * k + 28 * c + 24) if mixed else (84 + 4 * k + 52 * c + 48)


def gather_bytes_per_particle(mixed, k, p, c):
    """Algorithmic HBM bytes per particle of one gather launch with the next step's kick
    and drift fused: own state in and out, the list and its mirror index, every pair
    record once (p interacting pair sides, c contact sides per particle)."""
    vec = 12 if mixed else 24
    own_in = 24 + 8 + 48 + 4 + 8                           # x, a, v, w, id, displacement bound
    own_out = 24 + 48 + 8 + (24 if mixed else 0)           # x, v, w, bound (+ FP32 copies)
    return own_in + own_out + 4 * k + k + vec * p / 2 + vec * c / 2


def counter_record(mixed, stats, n):
    """The committed counter summary of the pair kernel, if it was taken from the current kernel
    source in the launch configuration (lanes per particle, form, skin, cell size) and size of
    the timed run; else None.  The summary holds `key = value` lines."""
    import hashlib
    try:
        rec = {}
        for line in open(COUNTER_FILE):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                rec[k.strip()] = v.strip()
        sha = hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    pre = "mixed" if mixed else "fp64"
    try:
        ok = (rec["kernel_source_sha1"] == sha and int(rec["n"]) == n
              and int(rec[pre + "_lanes"]) == stats["lanes"]
              and int(rec[pre + "_occupancy_form"]) == stats["occupancy_form"]
              and abs(float(rec[pre + "_skin"]) - stats["skin"]) < 1e-12
              and abs(float(rec[pre + "_cell_factor"]) - stats["cell_factor"]) < 1e-12)
    except (KeyError, ValueError):
        return None
    if not ok:
        return None
    return {"traffic": float(rec[pre + "_k_half_bytes"]), "valu_busy_frac": float(rec[pre + "_k_half_valu_busy_frac"]),
            "source": os.path.relpath(COUNTER_FILE, ROOT)}


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


def tuned_config(P, st, precision):
    """The configuration timed here: launch and list parameters (lanes per particle, kernel
    form, skin, cell size) left to the tuner."""
    return P.Config(box=st["L"], precision=precision, skin=-1.0, cell_factor=-1.0, lanes=0, **st["params"])


def run_gpu(P, st, precision, steps, warmup, prof_steps, say):
    """Creates a handle, runs warmup steps, times `steps` steps (HIP graphs, inputs resident),
    then a profiled pass of the same launch sequence for per-kernel times.  Returns the handle
    (for the shadow states) and the measurements."""
    import torch
    sim = P.Sim(tuned_config(P, st, precision), st["radii"], st["x"], st["v"], st["w"])
    sim.step(warmup)
    sim.stress_series()
    sim.reset_stress()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ser = sim.stress_series()
    stats = sim.stats()
    drag = sim.stress(0, P.STRESS_DRAG)[0, 1]
    mean = sim.stress(0, P.STRESS_TOTAL, P.STRESS_MEAN)[0, 1]
    sim.profile(True)
    sim.step(prof_steps)
    stage = [sim.stage_time(k) for k in range(3)]
    sim.profile(False)
    p = st["params"]
    n_l = max(stage[1][0], 1)
    say(f"  precision {precision}: {len(st['radii']) * steps / (t1 - t0):.3e} particle-steps/s, pair kernel "
        f"{stage[1][1] / n_l * 1e3:.1f} us, gather {stage[2][1] / n_l * 1e3:.1f} us")
    return sim, dict(seconds=t1 - t0, stats=stats, eta_mean=mean / (p["eta"] * p["gammadot"]),
                     eta_series=eta_r(ser, p["gammadot"], p["eta"], drag), pair_ms=stage[1][1] / n_l,
                     gather_ms=stage[2][1] / n_l, integrate_ms=stage[0][1] / max(stage[0][0], 1),
                     launches=stage[1][0])


def roofline(r, mixed, n):
    """Roofline object of the dominant kernel (the pair kernel): algorithmic bytes per launch
    (scope-table formula x N) over its average duration (HIP events on the library stream,
    profiled pass of the timed launch sequence), against 8 TB/s."""
    st = r["stats"]
    k, p, c = st["neighbours_per_particle"], st["interacting_per_particle"], st["contacts_per_particle"]
    bpp = pair_bytes_per_particle(mixed, k, c)
    achieved = bpp * n / (r["pair_ms"] * 1e-3) / 1e9
    rec = counter_record(mixed, st, n)
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": None if rec is None else rec["traffic"],
           "kernel": "k_half<%s>" % ("true" if mixed else "false"), "kernel_ms": r["pair_ms"],
           "bytes_per_particle": bpp, "algorithmic_bytes_per_launch": bpp * n,
           "list_per_particle": k, "interacting_per_particle": p, "contacts_per_particle": c}
    if rec is not None:
        # the kernel is bound by load latency and VALU issue rather than by HBM: its VALU-busy
        # fraction of 256 CUs x 4 SIMDs x 2.4 GHz, from the counter pass of the committed summary
        out["alu"] = {"bound": "alu", "valu_busy_frac": rec["valu_busy_frac"], "source": rec["source"]}
    gb = gather_bytes_per_particle(mixed, k, p, c)
    out["gather"] = {"kernel": "k_gather<%s>" % ("true" if mixed else "false"), "kernel_ms": r["gather_ms"],
                     "bytes_per_particle": gb, "frac": gb * n / (r["gather_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def host_cpu():
    """Model name and core counts of the host (the oracle runs on one of its cores)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(st, seconds_target=15.0):
    """The FP64 oracle as it stands, single-threaded on the host, on a bounded prefix of the same
    workload: steps of the same state after 2 warm-up steps, each step timed; the spread of
    the per-step times checks that the rate is constant over the prefix."""
    import numpy as np
    from oracle import oracle as O
    o = O.Oracle(O.Params(L=st["L"], **st["params"], flags=O.CELLS), st["radii"], st["x"], st["v"], st["w"])
    n = len(st["radii"])
    t0 = time.perf_counter()
    o.step(2)
    per = (time.perf_counter() - t0) / 2
    k = max(3, int(seconds_target / max(per, 1e-6)))
    ts = []
    for _ in range(k):
        t0 = time.perf_counter()
        o.step(1)
        ts.append(time.perf_counter() - t0)
    el = float(sum(ts))
    cv = float(np.std(ts) / np.mean(ts))
    return dict(value=n * k / el, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"{k} steps of the same {n}-particle workload after 2 warm-up steps, single thread, FP64, "
                       f"cell list rebuilt every step ({el:.1f} s; per-step time varies by {100 * cv:.1f}% "
                       f"(coefficient of variation), so the rate is constant over the prefix)",
                host_cpu=host_cpu(), per_step_cv=cv)


def eta_now(sim, P, r, gd, eta):
    """Relative viscosity of the last evaluation of replica r (contact + lubrication + drag, Sec. IV.D)."""
    return sim.stress(r, P.STRESS_TOTAL, P.STRESS_LAST)[0, 1] / (eta * gd)


def shadow_states(P, st, traj, nstates, every, say):
    """Shadow protocol: the FP64 handle `traj` advances; every `every` steps its state (positions,
    velocities, springs, offset, step counter) is evaluated by an FP64 and a mixed-precision
    handle, and the relative difference of eta_r at identical states is recorded."""
    import numpy as np
    p = st["params"]
    gd, eta = p["gammadot"], p["eta"]
    probe64 = P.Sim(tuned_config(P, st, P.FP64), st["radii"], st["x"], st["v"], st["w"])
    probe32 = P.Sim(tuned_config(P, st, P.MIXED), st["radii"], st["x"], st["v"], st["w"])
    e64, e32 = [], []
    for k in range(nstates):
        if k:
            traj.step(every)
        s = traj.get_state()
        cij, cs, _ = traj.contacts()
        for pr, acc in ((probe64, e64), (probe32, e32)):
            pr.set_state(0, s["x"], s["v"], s["w"], s_le=s["s_le"], step=s["step"], contacts=(cij, cs))
            acc.append(eta_now(pr, P, 0, gd, eta))
        say(f"  shadow state {k + 1} (step {s['step']}): eta_r FP64 {e64[-1]:.10g} mixed {e32[-1]:.10g}")
    probe64.close()
    probe32.close()
    e64, e32 = np.array(e64), np.array(e32)
    rel = (e32 - e64) / np.abs(e64)
    return {"states": int(nstates), "every_steps": every, "eta_r_fp64": e64.tolist(),
            "eta_r_rel_err_max": float(np.abs(rel).max()),
            "eta_r_mean_rel_err": float((e32.mean() - e64.mean()) / abs(e64.mean())),
            "target": 1e-4, "within_target": bool(np.abs(rel).max() <= 1e-4)}


def pair_time(sim, steps=100):
    """Average pair-kernel duration (ms) over `steps` steps, HIP events on the library stream."""
    sim.profile(True)
    sim.step(steps)
    launches, ms = sim.stage_time(1)
    sim.profile(False)
    return ms / max(launches, 1)


def hbm_frac(stats, mixed, n, ms):
    """Fraction of the HBM roofline of the pair kernel from its algorithmic bytes."""
    bpp = pair_bytes_per_particle(mixed, stats["neighbours_per_particle"], stats["contacts_per_particle"])
    return bpp * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS


def run_mixed_vs_fp64(P, st, steps, sample_every, say):
    """One workload in FP64 and in mixed precision from the same state and seed.

    Viscosity error, two protocols:
      * shadow: every `sample_every` steps the FP64 trajectory's state is injected into an
        FP64 and a mixed handle, which evaluate it; the relative difference of eta_r at
        identical states is recorded, and of its mean over the samples;
      * free-running: both precisions integrate independently; the difference of the mean
        eta_r over the run is compared with its block standard error.
    """
    import numpy as np
    import torch
    p = st["params"]
    gd, eta = p["gammadot"], p["eta"]
    n = len(st["radii"])
    traj = P.Sim(tuned_config(P, st, P.FP64), st["radii"], st["x"], st["v"], st["w"])
    say(f"  handles ready (n={n})")
    nst = max(steps // sample_every, 2)
    traj.step(sample_every)   # the first chunk also captures the step graphs (not timed)
    shadow = shadow_states(P, st, traj, nst, sample_every, say)
    done = nst * sample_every
    drag = traj.stress(0, P.STRESS_DRAG)[0, 1]
    ser64 = eta_r(traj.stress_series()[-done:], gd, eta, drag)
    st64 = traj.stats()
    # FP64 rate: sample_every further steps of the same trajectory, graphs already captured
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    traj.step(sample_every)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    ms64 = pair_time(traj)
    traj.close()
    free = P.Sim(tuned_config(P, st, P.MIXED), st["radii"], st["x"], st["v"], st["w"])
    free.step(sample_every)   # first chunk: graph capture (not timed); the run's series covers it
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    free.step(done - sample_every)
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    ser32 = eta_r(free.stress_series()[-done:], gd, eta, drag)
    st32 = free.stats()
    ms32 = pair_time(free)
    free.close()
    say("  mixed free run done")
    se = float(np.hypot(block_se(ser64), block_se(ser32)))
    m64, m32 = float(ser64.mean()), float(ser32.mean())
    return {
        "fp64": {"value": n * sample_every / t64, "pair_kernel_ms": ms64, "hbm_frac": hbm_frac(st64, False, n, ms64),
                 "lanes": st64["lanes"], "occupancy_form": st64["occupancy_form"], "skin": st64["skin"],
                 "rebuilds": st64["rebuilds"], "eta_r_mean": m64},
        "mixed": {"value": n * (done - sample_every) / t32, "pair_kernel_ms": ms32, "hbm_frac": hbm_frac(st32, True, n, ms32),
                  "lanes": st32["lanes"], "skin": st32["skin"], "rebuilds": st32["rebuilds"], "eta_r_mean": m32},
        "shadow": shadow,
        "free_running": {"eta_r_rel_diff": (m32 - m64) / abs(m64), "std_err_rel": se / abs(m64),
                         "within_3_se": bool(abs(m32 - m64) <= 3 * se)},
        "contacts_per_particle": st64["contacts_per_particle"], "sliding_fraction": st64["sliding_fraction"],
        "list_per_particle": st64["neighbours_per_particle"],
    }


def bench_c3_all(P, gen, steps, sample_every, say):
    out = {}
    for pe in (0.1, 10.0, 1000.0):
        wl = gen.Workload(f"bidisperse N=1000000 phi=0.56 Pe={pe:g}", 1_000_000, 0.56, pe, steps=steps)
        st = gen.make_state(wl)
        say(f"workload ready: {wl.name}")
        out[f"Pe={pe:g}"] = run_mixed_vs_fp64(P, st, steps, sample_every, say)
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
        cfgs = [tuned_config(P, s, prec) for s in sts]
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
                     "lanes": stt["lanes"], "occupancy_form": stt["occupancy_form"], "skin_replica0": stt["skin"],
                     "cell_factor": stt["cell_factor"], "tune_source": stt["tune_source"],
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
        h = P.Sim(tuned_config(P, s, P.MIXED), s["radii"], s["x"], s["v"], s["w"])
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
    sim = P.Sim(tuned_config(P, st, P.MIXED), st["radii"], st["x"], st["v"], st["w"])
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
            "lanes": stt["lanes"], "skin": stt["skin"], "cell_factor": stt["cell_factor"],
            "contacts_per_particle": stt["contacts_per_particle"], "sliding_fraction": stt["sliding_fraction"],
            "max_overlap": stt["max_overlap"], "rebuilds": stt["rebuilds"],
            "stress_total_mean": S.tolist(), "eta_r_mean": S[0, 1] / (p["eta"] * p["gammadot"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--prof-steps", type=int, default=200)
    ap.add_argument("--shadow-states", type=int, default=4, help="states of the shadow protocol (at least 1)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "c3-all", "sweep", "large"],
                    help="c3: 1,000,000 spheres, phi 0.56, Pe 10 (headline); c2: 50,000 spheres, phi 0.55; "
                         "c3-all: 1,000,000 spheres, mixed vs FP64 at Pe 0.1, 10, 1000 (long); "
                         "sweep: 64 batched replicas; large: 4,000,000 log-normal spheres")
    ap.add_argument("--sample-every", type=int, default=250, help="c3-all: steps between shadow samples")
    ap.add_argument("--trace", action="store_true",
                    help="profiling mode: a 256 MiB elementwise kernel (the calibration of the byte counters), "
                         "then --steps steps of the workload in FP64 and in mixed precision with the launch "
                         "parameters the tuner picks (cached in --tune-cache)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2307_13802_amd", "tune_cache_mi355x.json"),
                    help="file of tuned launch and list parameters (default: the parameters the tuner measured for "
                         "these workloads on an MI355X; a workload or device not in it is tuned at creation)")
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
    if args.tune_cache:
        P.set_tune_cache(args.tune_cache)
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
        for prec in (P.FP64, P.MIXED):
            sim = P.Sim(tuned_config(P, st, prec), st["radii"], st["x"], st["v"], st["w"])
            stt = sim.stats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(args.steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            sim.close()
            say(f"precision={prec} lanes={stt['lanes']} occupancy_form={stt['occupancy_form']} skin={stt['skin']:.4g} "
                f"cell_factor={stt['cell_factor']:.4g} tune_source={stt['tune_source']}: {args.steps} steps, "
                f"{len(st['radii']) * args.steps / el:.3e} particle-steps/s")
        return
    if args.workload in ("c3-all", "sweep", "large"):
        if args.workload == "c3-all":
            res = {"workload": "bidisperse N=1000000 phi=0.56, Pe in {0.1, 10, 1000}, mixed vs FP64",
                   "steps": args.steps, "results": bench_c3_all(P, gen, args.steps, args.sample_every, say)}
        elif args.workload == "sweep":
            res = {"workload": "64 replicas, N in [2000, 20000], phi in {0.45, 0.50, 0.54, 0.58}, "
                               "Pe log-spaced 1e-2..1e3, seeds 0..63",
                   "steps": args.steps, "results": bench_sweep(P, gen, args.steps, args.warmup, say)}
        else:
            res = bench_large(P, gen, args.steps, args.warmup, say)
        res["unit"] = "particle-steps/s"
        print(json.dumps(res), flush=True)
        return

    wl = gen.C3 if args.workload == "c3" else gen.C2
    st = gen.make_state(wl)
    n = len(st["radii"])
    name = f"bidisperse N={n} phi={wl.phi:g} Pe={wl.pe:g}"
    say(f"workload ready: {name}")
    sim64, f64 = run_gpu(P, st, P.FP64, args.steps, args.warmup, args.prof_steps, say)
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
        "data": "synthetic: seeded relaxed bidisperse packing (stands in for the paper's packings)",
        "config": {"workload": name, "n": n, "phi": wl.phi, "pe": wl.pe, "gammadot": st["params"]["gammadot"],
                   "kT": st["params"]["kT"], "mu": wl.mu, "dt": wl.dt, "hip_graph": True, "track_displacement": False,
                   "lanes_per_particle": f64["stats"]["lanes"], "occupancy_form": f64["stats"]["occupancy_form"],
                   "skin": f64["stats"]["skin"], "cell_factor": f64["stats"]["cell_factor"],
                   "tune_source": f64["stats"]["tune_source"]},
        "roofline": roofline(f64, False, n),
        "eta_r_fp64": f64["eta_mean"],
        "kernel_ms": {"pair": f64["pair_ms"], "gather": f64["gather_ms"], "integrate": f64["integrate_ms"]},
    }
    if not args.no_mixed:
        sim32, mix = run_gpu(P, st, P.MIXED, args.steps, args.warmup, args.prof_steps, say)
        sim32.close()
        vm = n * args.steps / mix["seconds"]
        se = np.hypot(block_se(f64["eta_series"]), block_se(mix["eta_series"]))
        out["mixed"] = {"value": vm, "ms_per_step": mix["seconds"] * 1e3 / args.steps,
                        "dtype": "f32 pair arithmetic, f64 positions / gaps / stress / integration",
                        "lanes_per_particle": mix["stats"]["lanes"], "occupancy_form": mix["stats"]["occupancy_form"],
                        "skin": mix["stats"]["skin"], "cell_factor": mix["stats"]["cell_factor"],
                        "speedup_vs_fp64": vm / value, "roofline": roofline(mix, True, n),
                        "kernel_ms": {"pair": mix["pair_ms"], "gather": mix["gather_ms"]},
                        "eta_r": mix["eta_mean"],
                        "eta_r_rel_diff_free_running": (mix["eta_mean"] - f64["eta_mean"]) / f64["eta_mean"],
                        "eta_r_diff_std_err": float(se / abs(f64["eta_mean"]))}
        say("shadow protocol")
        out["mixed"]["shadow"] = shadow_states(P, st, sim64, max(1, args.shadow_states), 50, say)
    sim64.close()
    if not args.no_cpu:
        say("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(st)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
