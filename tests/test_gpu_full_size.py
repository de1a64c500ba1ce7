"""GPU parity at the benchmark's full sizes, on relaxed packings, through the C ABI.

* 1,000,000 bidisperse spheres, phi = 0.56, Pe = 10, FP64, in the launch
  configuration the benchmark times (tuned lanes, kernel form, skin and cell
  size): the whole interaction set and contact table bit-exact, every force and
  torque, all five stresses and eta_r against the FP64 oracle, at creation and
  after two steps.
* The same workload under the shadow protocol: an FP64 trajectory whose states
  are evaluated by an FP64 and a mixed-precision handle; eta_r of mixed against
  FP64 within 1e-4 at every state, and the FP64 value against the oracle's.
* The 64-replica flow-curve sweep (N in [2000, 20000], four volume fractions,
  Pe from 1e-2 to 1e3, seeds 0..63) in one handle, mixed precision: every
  replica bit-identical to the same replica run alone.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from inputs import gen

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-10
TOL_ETA_MIXED = 1e-4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_13802_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def c3():
    _say("packing the 1,000,000-sphere workload (phi = 0.56)")
    return gen.make_state(gen.C3)


def _bench_cfg(P, st, precision):
    """The configuration the benchmark times: everything tunable left to the tuner."""
    return P.Config(box=st["L"], precision=precision, skin=-1.0, cell_factor=-1.0, lanes=0, **st["params"])


def _compare(P, sim, orc, label, exact_springs=True):
    p = sim.configs[0]
    pg, po = sim.pairs(), orc.pairs()
    cg, co = sim.contacts(), orc.contacts()
    Fg, Tg = sim.forces()
    so = orc.state()
    Fa, Ta = orc.norms()
    ef = float((np.linalg.norm(Fg - so["F"], axis=1) / Fa).max())
    et = float((np.linalg.norm(Tg - so["T"], axis=1) / np.maximum(Ta, 1e-300)).max())
    Sg = np.stack([sim.stress(0, c, P.STRESS_LAST) for c in range(5)])
    So = orc.stress_all()
    es = float((np.abs(Sg - So).reshape(5, 9).max(axis=1) / np.abs(So).reshape(5, 9).max(axis=1)).max())
    eg, eo = Sg[4][0, 1] / (p.eta * p.gammadot), orc.eta_r()
    _say(f"  {label}: pairs {len(pg)}/{len(po)} contacts {len(cg[0])}/{len(co[0])} F err {ef:.2e} "
         f"T err {et:.2e} stress err {es:.2e} eta_r {eg:.10g} / {eo:.10g}")
    assert np.array_equal(pg, po)
    assert np.array_equal(cg[0], co[0])
    if exact_springs:   # from an identical state: the same bits
        assert np.array_equal(cg[1], co[1]) and np.array_equal(cg[2], co[2])
    else:               # after steps the positions differ in the last bits (force sums in another order)
        assert np.abs(cg[1] - co[1]).max() <= 1e-9 * np.abs(co[1]).max()
    assert ef <= TOL_F64 and et <= TOL_F64 and es <= TOL_F64
    assert abs(eg - eo) <= TOL_F64 * abs(eo)


def test_c3_relaxed_fp64_matches_oracle(P, c3):
    st = c3
    _say("case: N=1000000 phi=0.56 Pe=10 FP64, tuned launch, creation and 2 steps against the oracle")
    sim = P.Sim(_bench_cfg(P, st, P.FP64), st["radii"], st["x"], st["v"], st["w"])
    stt = sim.stats()
    _say(f"  tuned: lanes {stt['lanes']} form {stt['occupancy_form']} skin {stt['skin']:.3f} "
         f"cell {stt['cell_factor']} (source {stt['tune_source']})")
    orc = O.Oracle(O.Params(L=st["L"], **st["params"], flags=O.CELLS), st["radii"], st["x"], st["v"], st["w"])
    _compare(P, sim, orc, "creation")
    sim.step(2)
    orc.step(2)
    g, o = sim.get_state(), orc.state()
    dx = float(np.abs(g["x"] - o["x"]).max())
    _say(f"  after 2 steps: max |dx| {dx:.2e}")
    assert g["step"] == o["step"] and g["s_le"] == o["s_le"] and dx < 1e-12
    _compare(P, sim, orc, "step 2", exact_springs=False)
    # and from the oracle's state injected into the library, one evaluation: bit-exact again
    cij, cs, _ = orc.contacts()
    sim.set_state(0, o["x"], o["v"], o["w"], s_le=o["s_le"], step=o["step"], contacts=(cij, cs))
    del orc
    ref = O.Oracle(O.Params(L=st["L"], **st["params"], flags=O.CELLS), st["radii"], o["x"], o["v"], o["w"],
                   s_le=o["s_le"], step=o["step"], contacts=(cij, cs))
    _compare(P, sim, ref, "injected state at step 2")
    sim.close()


def test_c3_shadow_viscosity_mixed_within_1e4(P, c3):
    """Shadow protocol on 1,000,000 spheres: every 100 steps of an FP64 trajectory, its state
    (positions, velocities, springs, offset, step counter) is evaluated by an FP64 and a
    mixed-precision handle; |eta_r(mixed) - eta_r(FP64)| / eta_r(FP64) <= 1e-4 at each of
    4 states, and at the first the FP64 eta_r equals the oracle's evaluation of that state."""
    st = c3
    p = st["params"]
    traj = P.Sim(_bench_cfg(P, st, P.FP64), st["radii"], st["x"], st["v"], st["w"])
    probe64 = P.Sim(_bench_cfg(P, st, P.FP64), st["radii"], st["x"], st["v"], st["w"])
    probe32 = P.Sim(_bench_cfg(P, st, P.MIXED), st["radii"], st["x"], st["v"], st["w"])
    rel = []
    for k in range(4):
        traj.step(100)
        s = traj.get_state()
        cij, cs, _ = traj.contacts()
        eta = []
        for pr in (probe64, probe32):
            pr.set_state(0, s["x"], s["v"], s["w"], s_le=s["s_le"], step=s["step"], contacts=(cij, cs))
            eta.append(pr.stress(0, P.STRESS_TOTAL, P.STRESS_LAST)[0, 1] / (p["eta"] * p["gammadot"]))
        rel.append((eta[1] - eta[0]) / abs(eta[0]))
        _say(f"case: shadow state {k + 1} (step {s['step']}): eta_r FP64 {eta[0]:.10g} mixed {eta[1]:.10g} "
             f"rel {rel[-1]:.2e}")
        if k == 0:
            orc = O.Oracle(O.Params(L=st["L"], **p, flags=O.CELLS), st["radii"], s["x"], s["v"], s["w"],
                           s_le=s["s_le"], step=s["step"], contacts=(cij, cs))
            _say(f"  oracle eta_r {orc.eta_r():.10g}")
            assert abs(eta[0] - orc.eta_r()) <= TOL_F64 * abs(orc.eta_r())
            del orc
    for h in (traj, probe64, probe32):
        h.close()
    assert max(abs(r) for r in rel) <= TOL_ETA_MIXED


def test_c4_sweep_64_replicas_match_single(P):
    """The flow-curve sweep of 64 replicas in one handle, mixed precision, 30 steps: every
    replica's state, forces and stress series bit-identical to the same replica alone."""
    wls = gen.sweep_replicas(64)
    sts = []
    for r, wl in enumerate(wls):
        sts.append(gen.make_state(wl))
        if r % 16 == 15:
            _say(f"  packed {r + 1}/64 sweep replicas")
    cfgs = [P.Config(box=s["L"], precision=P.MIXED, lanes=1, **s["params"]) for s in sts]
    ntot = sum(len(s["radii"]) for s in sts)
    _say(f"case: 64 sweep replicas ({ntot} spheres) batched vs alone, 30 steps, mixed")
    multi = P.Sim(cfgs, [s["radii"] for s in sts], [s["x"] for s in sts], [s["v"] for s in sts],
                  [s["w"] for s in sts])
    multi.step(30)
    for k, s in enumerate(sts):
        one = P.Sim(cfgs[k], s["radii"], s["x"], s["v"], s["w"])
        one.step(30)
        a, b = multi.get_state(k), one.get_state()
        for key in ("x", "v", "w", "F", "T"):
            assert np.array_equal(a[key], b[key]), (k, key)
        assert np.array_equal(multi.stress_series(k), one.stress_series()), k
        assert multi.stats(k)["rebuilds"] >= 1
        one.close()
    _say("  all 64 replicas bit-identical")
    multi.close()
