"""GPU parity: the HIP path, called through the C ABI, against the FP64 CPU oracle.

Bars: neighbour sets and contact springs bit-exact (FP64); forces and torques
within 1e-10 relative to the per-particle sum of pair-force norms; stresses
within 1e-10 relative; mixed precision within its FP32 bound.
"""
import math
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from inputs import gen

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-10
# mixed: FP32 pair arithmetic (unit roundoff 6e-8) with hardware log/sin/cos;
# forces carry ~1e-6 relative error per pair, Brownian terms a few 1e-6
TOL_MIX = 5e-5


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


def _cfg(P, st, precision=0, flags=0, **kw):
    p = dict(st["params"])
    p.update(kw)
    return P.Config(box=st["L"], precision=precision, flags=flags, **p)


def _state(n=500, phi=0.5, pe=1.0, kT=1.0, seed=0, mu=0.5):
    w = gen.Workload("t", n, phi, pe, kT=kT, seed=seed, mu=mu)
    return gen.make_state(w)


def _force_err(Fg, Fo, norm):
    e = np.linalg.norm(Fg - Fo, axis=1) / np.maximum(norm, 1e-300)
    return float(e.max())


def _stress_err(Sg, So):
    Sg = np.asarray(Sg).reshape(3, 9)
    So = np.asarray(So).reshape(3, 9)
    out = []
    for c in range(3):
        scale = max(np.abs(So[c]).max(), 1e-300)
        out.append(float(np.abs(Sg[c] - So[c]).max() / scale))
    return max(out)


def _gpu_stress27(sim, r=0):
    import paper_2307_13802_amd as P
    return np.stack([sim.stress(r, c, P.STRESS_LAST) for c in (P.STRESS_CONTACT, P.STRESS_LUB, P.STRESS_BROWN)])


def _compare_eval(P, sim, orc, tol, exact=True, r=0):
    Fg, Tg = sim.forces(r)
    so = orc.state()
    Fa, Ta = orc.norms()
    ef = _force_err(Fg, so["F"], Fa)
    et = _force_err(Tg, so["T"], np.maximum(Ta, 1e-300))
    pg, po = sim.pairs(r), orc.pairs()
    cg, co = sim.contacts(r), orc.contacts()
    es = _stress_err(_gpu_stress27(sim, r), orc.stress())
    _say(f"  F err {ef:.2e}  T err {et:.2e}  stress err {es:.2e}  pairs {len(pg)}/{len(po)}  contacts {len(cg[0])}/{len(co[0])}")
    assert np.array_equal(pg, po)
    assert np.array_equal(cg[0], co[0])
    if exact:
        assert np.array_equal(cg[1], co[1]), np.abs(cg[1] - co[1]).max()
        assert np.array_equal(cg[2], co[2])
    else:
        scale = max(np.abs(co[1]).max(), 1e-30)
        assert np.abs(cg[1] - co[1]).max() <= 1e-4 * scale
    assert ef <= tol and et <= tol and es <= tol
    return ef, et, es


def test_create_fp64_matches_oracle(P):
    _say("case: create N=500 phi=0.5 FP64, forces at the initial state")
    st = _state()
    sim = P.Sim(_cfg(P, st), st["radii"], st["x"], st["v"], st["w"])
    orc = O.Oracle(O.Params(L=st["L"], **st["params"]), st["radii"], st["x"], st["v"], st["w"])
    _compare_eval(P, sim, orc, TOL_F64)
    # Verlet set at the same positions with the same skin, bit-exact
    assert np.array_equal(sim.nlist(), orc.verlet_pairs(0.2))


def test_injected_contacts_and_offset(P):
    """Random stored springs on every overlapping pair, Lees-Edwards offset, shear: one evaluation."""
    rng = np.random.default_rng(3)
    n = 200
    L = (14.0, 13.0, 15.0)
    a = gen.radii_bidisperse(n, 4)
    x, v, w = gen.random_state(n, L, a, seed=11, kT=0.5, gammadot=0.4)
    for s_le in (0.0, L[0] / 3.0, L[0] - 1e-9):
        _say(f"case: random overlapping state n={n} s_le={s_le:.6f}")
        prm = dict(rho=0.1, eta=0.1, kn=1e4, kt=2e4 / 7, mu=0.5, kT=0.5, gammadot=0.4, dt=1e-4, xi_cut=0.05,
                   xi_min=1e-3, seed=99)
        probe = O.Oracle(O.Params(L=L, **prm), a, x, v, w, s_le=s_le)
        # overlapping pairs (the oracle's contact list after its evaluation) get random springs
        cij = probe.contacts()[0]
        cs = rng.normal(size=(len(cij), 3)) * 1e-3
        orc = O.Oracle(O.Params(L=L, **prm), a, x, v, w, s_le=s_le, contacts=(cij, cs))
        cfg = P.Config(box=L, **prm, max_overlap=10.0)
        sim = P.Sim(cfg, a, x, v, w)
        sim.set_state(0, x, v, w, s_le=s_le, step=0, contacts=(cij, cs))
        _compare_eval(P, sim, orc, TOL_F64)


def test_verlet_lists_every_layout_match_brute_force(P):
    """The list build against the oracle's O(N^2) search, bit-exact, over cell sizes, skins,
    Lees-Edwards offsets and boxes with 3 cells or 1 cell (every x cell searched) along a side."""
    n = 200
    a = gen.radii_bidisperse(n, 4)
    prm = dict(rho=0.1, eta=0.1, kn=1e4, kt=2e4 / 7, mu=0.5, kT=0.5, gammadot=0.4, dt=1e-4, xi_cut=0.05,
               xi_min=1e-3, seed=99)
    for L in ((14.0, 13.0, 15.0), (20.0, 9.5, 20.0), (7.2, 20.0, 18.0)):
        x, v, w = gen.random_state(n, L, a, seed=5, kT=0.5, gammadot=0.4)
        for skin in (0.1, 0.6):
            for cf in (1.0, 1.5, 2.0, 3.0):
                sim = P.Sim(P.Config(box=L, **prm, max_overlap=10.0, skin=skin, cell_factor=cf, lanes=1), a, x, v, w)
                stt = sim.stats()
                for s_le in (0.0, L[0] / 3.0, L[0] - 1e-9):
                    sim.set_state(0, x, v, w, s_le=s_le, step=0)
                    orc = O.Oracle(O.Params(L=L, **prm), a, x, v, w, s_le=s_le)
                    ref = orc.verlet_pairs(skin)
                    got = sim.nlist()
                    ok = np.array_equal(got, ref)
                    if not ok or s_le == 0.0:
                        _say(f"case: box {L} skin {skin} cell factor {cf} cells "
                             f"{stt['cells_x']}x{stt['cells_y']}x{stt['cells_z']} s_le {s_le:.4f}: "
                             f"{len(got)} / {len(ref)} pairs")
                    assert ok
                sim.close()


def _cut_boundary(x0, a1, a2, xi_cut):
    """The largest x with (x0 - x)^2 <= ((a1 + a2)(1 + xi_cut / 2))^2 in FP64, the range test's own arithmetic
    (Sec. II.B, cut-off inclusive), and the next double above it: the last position in range and the first out."""
    rc = (a1 + a2) * (1.0 + 0.5 * xi_cut)
    inside = lambda x: (x0 - x) * (x0 - x) <= rc * rc
    x = x0 + rc
    while inside(x):
        x = float(np.nextafter(x, np.inf))
    while not inside(x):
        x = float(np.nextafter(x, -np.inf))
    return x, float(np.nextafter(x, np.inf))


def test_adversarial_pairs(P):
    """Hand-built pairs, each far from the others: one exactly at the cut-off (in range), one an ulp beyond it,
    one at a gap far below xi_min (the regularised lubrication), one in shallow contact across the sheared
    y boundary, and one in contact across the x boundary; offsets 0, L/3 and L minus 1e-9."""
    L = (30.0, 30.0, 30.0)
    prm = dict(rho=0.1, eta=0.1, kn=1e4, kt=2e4 / 7, mu=0.5, kT=0.5, gammadot=0.4, dt=1e-4, xi_cut=0.05,
               xi_min=1e-3, seed=5)
    x_in, x_out = _cut_boundary(5.0, 1.0, 1.4, prm["xi_cut"])
    rng = np.random.default_rng(12)
    for s_le in (0.0, L[0] / 3.0, L[0] - 1e-9):
        a = np.array([1.0, 1.4, 1.0, 1.4, 1.0, 1.0, 1.4, 1.0, 1.0, 1.4])
        x = np.array([
            [5.0, 5.0, 5.0], [x_in, 5.0, 5.0],                       # gap exactly at the cut-off: in range
            [5.0, 15.0, 5.0], [x_out, 15.0, 5.0],                    # an ulp beyond: out of range
            [15.0, 5.0, 20.0], [15.0 + 2.0 + 1e-6, 5.0, 20.0],       # gap 1e-6 << xi_min
            [12.0, 0.3, 12.0], [(12.0 + s_le) % L[0], L[1] - 2.09, 12.0],  # contact through y = 0 / Ly
            [0.2, 20.0, 25.0], [L[0] - 1.9, 20.0, 25.0],             # contact through x = 0 / Lx
        ])
        v = rng.normal(size=(10, 3)) * 0.3
        w = rng.normal(size=(10, 3)) * 0.3
        _say(f"case: adversarial pairs s_le={s_le:.9f} (cut-off at x={x_in!r}, first out {x_out!r})")
        orc = O.Oracle(O.Params(L=L, **prm), a, x, v, w, s_le=s_le)
        sim = P.Sim(P.Config(box=L, **prm, max_overlap=1.0), a, x, v, w)
        sim.set_state(0, x, v, w, s_le=s_le, step=0)
        _compare_eval(P, sim, orc, TOL_F64)
        pairs = {tuple(p) for p in np.asarray(sim.pairs()).tolist()}
        assert (0, 1) in pairs and (2, 3) not in pairs and (4, 5) in pairs
        assert (6, 7) in pairs and (8, 9) in pairs
        contacts = {tuple(c) for c in np.asarray(sim.contacts()[0]).tolist()}
        assert (6, 7) in contacts and (8, 9) in contacts and (4, 5) not in contacts


def test_step_trajectory_fp64(P):
    """Short trajectory: the same state after each step (chaos sets in only later)."""
    st = _state(n=500, phi=0.5)
    for flags in (0, P.REBUILD_EACH_STEP | P.NO_GRAPH):
        _say(f"case: trajectory N=500 flags={flags:#x}")
        sim = P.Sim(_cfg(P, st, flags=flags), st["radii"], st["x"], st["v"], st["w"])
        orc = O.Oracle(O.Params(L=st["L"], **st["params"]), st["radii"], st["x"], st["v"], st["w"])
        for k in range(4):
            sim.step(5)
            series = sim.stress_series()
            oser = orc.step(5, series=True)
            gs = sim.get_state()
            os_ = orc.state()
            dx = np.abs(gs["x"] - os_["x"]).max()
            dv = np.abs(gs["v"] - os_["v"]).max() / np.abs(os_["v"]).max()
            _say(f"  after {5 * (k + 1)} steps: |dx| {dx:.2e} |dv|/|v| {dv:.2e}")
            assert gs["step"] == os_["step"] and gs["s_le"] == os_["s_le"]
            assert dx < 1e-11 and dv < 1e-9
            assert series.shape[0] == 5
            assert _stress_err(series[-1], oser[-1].reshape(3, 3, 3)) < 1e-8
            assert np.array_equal(sim.contacts()[0], orc.contacts()[0])


@pytest.mark.parametrize("lanes, flags", [(1, 0x800), (2, 0x800), (4, 0x800), (1, 0x400), (2, 0x400), (4, 0x400)])
def test_pair_kernel_forms(P, lanes, flags):
    """Every launch shape of the pair kernel (1, 2 or 4 lanes per particle; in FP64 also its
    form for occupancy) gives the oracle's forces and exact springs."""
    st = _state(n=1500, phi=0.55, seed=7)
    for prec, tol, exact in ((P.FP64, TOL_F64, True), (P.MIXED, TOL_MIX, False)):
        if prec == P.MIXED and flags == P.HALF_OCC_ON:
            continue
        _say(f"case: lanes={lanes} flags={flags:#x} precision={prec} N=1500 phi=0.55")
        sim = P.Sim(_cfg(P, st, precision=prec, lanes=lanes, flags=flags), st["radii"], st["x"], st["v"], st["w"])
        stt = sim.stats()
        assert stt["lanes"] == lanes and stt["pair_kernel"] == P.KERNEL_HALF
        assert stt["occupancy_form"] == (1 if flags == P.HALF_OCC_ON else 0)
        orc = O.Oracle(O.Params(L=st["L"], **st["params"]), st["radii"], st["x"], st["v"], st["w"])
        _compare_eval(P, sim, orc, tol, exact=exact)


def test_launch_and_list_parameters_bit_identical(P):
    """Lanes per particle, the kernel form (with its queue in rounds of 2048 or of 64 items),
    the Verlet skin and the cell size of the layout change neither the interacting pairs nor
    the order in which each particle's terms are summed: whole trajectories agree bit for bit,
    in both precisions (the parameters the tuner chooses among)."""
    st = _state(n=2000, phi=0.55, seed=8)
    amin = float(st["radii"].min())
    for prec in (P.FP64, P.MIXED):
        runs = []
        cases = [(1, P.HALF_OCC_OFF, 0.0, 0.0), (2, P.HALF_OCC_OFF, 0.0, 0.0), (4, P.HALF_OCC_OFF, 0.0, 0.0),
                 (1, 0, 0.1 * amin, 0.0), (2, 0, 0.4 * amin, 2.0), (1, 0, 0.15 * amin, 1.5)]
        if prec == P.FP64:
            cases += [(1, P.HALF_OCC_ON, 0.0, 0.0), (2, P.HALF_OCC_ON, 0.3 * amin, 0.0), (4, P.HALF_OCC_ON, 0.0, 2.0),
                      (1, P.HALF_OCC_ON | P.SMALL_QUEUE, 0.0, 0.0), (2, P.HALF_OCC_ON | P.SMALL_QUEUE, 0.1 * amin, 1.0)]
        for lanes, flags, skin, cell in cases:
            _say(f"case: 60 steps precision={prec} lanes={lanes} flags={flags:#x} skin={skin:.3f} cell={cell}")
            sim = P.Sim(_cfg(P, st, precision=prec, lanes=lanes, flags=flags, skin=skin, cell_factor=cell),
                        st["radii"], st["x"], st["v"], st["w"])
            stt = sim.stats()
            assert stt["skin"] == (skin if skin > 0 else 0.2 * amin) and stt["cell_factor"] == (cell or 1.0)
            sim.step(60)
            runs.append(sim.get_state())
        for other in runs[1:]:
            for key in ("x", "v", "w", "F", "T"):
                assert np.array_equal(runs[0][key], other[key]), key


def test_tuner_cache_reused(P, tmp_path):
    """With skin, cell factor, lanes and form left to the tuner, the first creation measures
    them and writes the cache; a second creation of the same workload reads them back
    (tune_source 2) and reproduces the first run bit for bit, stresses included."""
    st = _state(n=3000, phi=0.55, seed=12)
    path = tmp_path / "tune.json"
    P.set_tune_cache(str(path))
    try:
        runs = []
        for k in range(2):
            _say(f"case: tuned creation {k} N=3000 phi=0.55")
            sim = P.Sim(_cfg(P, st, skin=-1.0, cell_factor=-1.0, lanes=0), st["radii"], st["x"], st["v"], st["w"])
            stt = sim.stats()
            _say(f"  tune_source {stt['tune_source']} lanes {stt['lanes']} form {stt['occupancy_form']} "
                 f"skin {stt['skin']:.3f} cell {stt['cell_factor']}")
            sim.step(50)
            runs.append((stt, sim.get_state(), sim.stress_series()))
            sim.close()
        (s1, a, sa), (s2, b, sb) = runs
        assert s1["tune_source"] == 1 and s2["tune_source"] == 2
        for key in ("lanes", "occupancy_form", "skin", "cell_factor", "cells_x"):
            assert s1[key] == s2[key], key
        for key in ("x", "v", "w", "F", "T"):
            assert np.array_equal(a[key], b[key]), key
        assert np.array_equal(sa, sb)
        txt = path.read_text()
        assert txt.startswith("{") and '"lanes"' in txt
    finally:
        P.set_tune_cache(None)


def test_planned_rebuilds_match_rebuild_every_step(P):
    """Host-planned list builds (with device-side expiry halts) give bit-identical trajectories
    to building the list at every step: no interacting pair is ever missing from a list."""
    st = _state(n=500, phi=0.5, kT=1.0)
    runs = []
    for flags in (0, P.REBUILD_EACH_STEP):
        _say(f"case: 400 steps N=500 kT=1 flags={flags:#x}")
        sim = P.Sim(_cfg(P, st, flags=flags, lanes=1), st["radii"], st["x"], st["v"], st["w"])
        for _ in range(4):
            sim.step(100)
        runs.append((sim.get_state(), sim.stats()))
    (a, sa), (b, sb) = runs
    _say(f"  rebuilds planned {sa['rebuilds']} vs every step {sb['rebuilds']}")
    assert sa["rebuilds"] < sb["rebuilds"]
    for key in ("x", "v", "w", "F", "T"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("prec", [0, 1])
def test_graphs_match_direct_launches(P, prec):
    """Steps through the chained HIP graphs (64, 8 and 1 steps handing over through the fused
    gather) are bit-identical to the same steps launched directly, including chunks that end
    in a list-expiry halt and resume after the rebuild (fast diffusion, kT = 1)."""
    st = _state(n=700, phi=0.5, kT=1.0, seed=21)
    runs = []
    for flags in (0, P.NO_GRAPH):
        _say(f"case: 2 x 150 steps precision={prec} flags={flags:#x}")
        sim = P.Sim(_cfg(P, st, precision=prec, flags=flags, lanes=1), st["radii"], st["x"], st["v"], st["w"])
        sim.step(150)
        sim.step(150)
        runs.append((sim.get_state(), sim.stats()))
    (a, sa), (b, sb) = runs
    _say(f"  list builds {sa['rebuilds']} / {sb['rebuilds']}")
    assert sa["rebuilds"] == sb["rebuilds"] and sa["rebuilds"] > 1
    for key in ("x", "v", "w", "F", "T"):
        assert np.array_equal(a[key], b[key]), key


def test_mixed_precision_create(P):
    _say("case: create N=500 mixed precision")
    st = _state()
    sim = P.Sim(_cfg(P, st, precision=P.MIXED), st["radii"], st["x"], st["v"], st["w"])
    orc = O.Oracle(O.Params(L=st["L"], **st["params"]), st["radii"], st["x"], st["v"], st["w"])
    _compare_eval(P, sim, orc, TOL_MIX, exact=False)


@pytest.mark.parametrize("pe", [0.1, 10.0])
def test_mixed_viscosity_shadow(P, pe):
    """The shadow protocol on a small system: eight states along an FP64 trajectory (5,000 bidisperse spheres,
    phi = 0.55) are evaluated by an FP64 and a mixed handle; the relative viscosity of each (contact +
    lubrication + drag shear stress over eta gammadot, Sec. II.E) and its mean agree within 1e-4.  (These are
    the first 400 steps from a relaxed packing: at Pe = 0.1, where gammadot is small, the values themselves swing
    widely, even in sign; the test compares the two precisions at identical states.)"""
    st = gen.make_state(gen.Workload("shadow", 5000, 0.55, pe, seed=3))
    p = st["params"]
    mk = lambda prec: P.Sim(P.Config(box=st["L"], precision=prec, **p), st["radii"], st["x"], st["v"], st["w"])
    traj, p64, p32 = mk(P.FP64), mk(P.FP64), mk(P.MIXED)
    _say(f"case: shadow protocol N=5000 phi=0.55 Pe={pe}, 8 states 50 steps apart")
    e64, e32 = [], []
    for _ in range(8):
        traj.step(50)
        s = traj.get_state()
        cij, cs, _ = traj.contacts()
        for pr, acc in ((p64, e64), (p32, e32)):
            pr.set_state(0, s["x"], s["v"], s["w"], s_le=s["s_le"], step=s["step"], contacts=(cij, cs))
            acc.append(pr.stress(0, P.STRESS_TOTAL, P.STRESS_LAST)[0, 1] / (p["eta"] * p["gammadot"]))
    e64, e32 = np.array(e64), np.array(e32)
    rel = np.abs(e32 - e64) / np.abs(e64)
    mean_rel = abs(e32.mean() - e64.mean()) / abs(e64.mean())
    _say(f"  eta_r FP64 {e64.mean():.6f}; mixed vs FP64: max rel {rel.max():.2e}, mean rel {mean_rel:.2e}")
    assert rel.max() <= 1e-4 and mean_rel <= 1e-4
    for h in (traj, p64, p32):
        h.close()


def test_ragged_and_tiny_systems(P):
    """A lone sphere (one-body terms only), one pair in contact, and sizes that leave
    ragged tiles: the first evaluation, then five steps, against the oracle."""
    for n, phi in ((1, 0.001), (2, 0.001), (37, 0.3), (257, 0.45), (1000, 0.55)):
        _say(f"case: ragged n={n} phi={phi}")
        w = gen.Workload("t", n, phi, 1.0, kT=1.0, seed=n)
        a = gen.radii_bidisperse(n, n)
        L = max(gen.box_length(a, phi), 2.0 * (2 * 1.4 * 1.025 + 0.2) + 0.1)
        x = gen.relaxed_positions(a, L, n)
        if n == 2:  # put the pair into contact
            x[1] = x[0] + np.array([a[0] + a[1] - 1e-3, 0.0, 0.0])
            x %= L
        _, v, om = gen.random_state(n, (L, L, L), a, seed=1)
        st = dict(radii=a, x=x, v=v, w=om, L=(L, L, L), params=w.params())
        sim = P.Sim(_cfg(P, st), a, x, v, om)
        orc = O.Oracle(O.Params(L=st["L"], **st["params"]), a, x, v, om)
        _compare_eval(P, sim, orc, TOL_F64)
        sim.step(5)
        orc.step(5)
        gs, os_ = sim.get_state(), orc.state()
        dx = np.abs(gs["x"] - os_["x"]).max()
        dv = np.abs(gs["v"] - os_["v"]).max() / np.abs(os_["v"]).max()
        _say(f"  after 5 steps: |dx| {dx:.2e} |dv|/|v| {dv:.2e}")
        assert gs["step"] == os_["step"] and gs["s_le"] == os_["s_le"]
        assert dx < 1e-11 and dv < 1e-9
        assert np.array_equal(sim.pairs(), orc.pairs())


def test_batched_replicas_match_single(P):
    """Replicas of uneven size in one handle: each bit-identical to the same replica run alone."""
    sts = [_state(n=n, phi=phi, seed=s) for n, phi, s in ((300, 0.45, 1), (777, 0.55, 2), (512, 0.5, 3))]
    # one lane per particle: each force is summed over the interacting partners in id order,
    # independent of when the (skin-padded) list was built
    cfgs = [_cfg(P, st, seed=10 + k, lanes=1) for k, st in enumerate(sts)]
    _say("case: 3 replicas batched vs alone, 30 steps")
    multi = P.Sim(cfgs, [s["radii"] for s in sts], [s["x"] for s in sts], [s["v"] for s in sts],
                  [s["w"] for s in sts])
    multi.step(30)
    for k, st in enumerate(sts):
        one = P.Sim(cfgs[k], st["radii"], st["x"], st["v"], st["w"])
        one.step(30)
        a, b = multi.get_state(k), one.get_state()
        _say(f"  replica {k}: max |dx| {np.abs(a['x'] - b['x']).max():.2e}")
        for key in ("x", "v", "w", "F", "T"):
            assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_sweep_replicas_match_single(P, prec):
    """Eight replicas of a flow-curve sweep in one handle (uneven N, four volume fractions, Pe from 1e-2 to 1e3,
    own seeds), half-pair kernel: each bit-identical to the same replica run alone, in both precisions."""
    spec = [(300, 0.45, 1e-2), (777, 0.50, 0.1), (512, 0.54, 1.0), (1200, 0.58, 10.0), (450, 0.45, 1e2),
            (900, 0.50, 1e3), (600, 0.54, 0.3), (1024, 0.58, 30.0)]
    sts = [gen.make_state(gen.Workload(f"sweep{k}", n, phi, pe, seed=20 + k)) for k, (n, phi, pe) in enumerate(spec)]
    # fixed launch parameters: the stress sums follow the launch shape (trajectories would agree anyway)
    cfgs = [P.Config(box=st["L"], precision=prec, pair_kernel=P.KERNEL_HALF, lanes=1, **st["params"]) for st in sts]
    _say(f"case: 8 sweep replicas batched vs alone, 25 steps, precision {prec}")
    multi = P.Sim(cfgs, [s["radii"] for s in sts], [s["x"] for s in sts], [s["v"] for s in sts],
                  [s["w"] for s in sts])
    multi.step(25)
    for k, st in enumerate(sts):
        one = P.Sim(cfgs[k], st["radii"], st["x"], st["v"], st["w"])
        one.step(25)
        a, b = multi.get_state(k), one.get_state()
        for key in ("x", "v", "w", "F", "T"):
            assert np.array_equal(a[key], b[key]), (k, key)
        assert np.array_equal(multi.stress_series(k), one.stress_series())
        one.close()
    multi.close()


@pytest.mark.parametrize("kernel, lanes", [(0, 1), (0, 2), (3, 1), (3, 4)])
def test_deterministic_and_restart(P, kernel, lanes):
    """Identical runs are bit-identical; a restart from get_state/contacts continues the
    run bit-identically (each particle's terms are summed in an order that does not depend
    on when the list was built)."""
    st = _state(n=600, phi=0.55, seed=5)
    cfg = _cfg(P, st, lanes=lanes, pair_kernel=kernel)
    _say(f"case: determinism and restart, 40 steps, kernel={kernel} lanes={lanes}")
    s1 = P.Sim(cfg, st["radii"], st["x"], st["v"], st["w"])
    s2 = P.Sim(cfg, st["radii"], st["x"], st["v"], st["w"])
    s1.step(40)
    s2.step(20)
    mid = s2.get_state()
    ij, cs, _ = s2.contacts()
    s2.step(20)
    s3 = P.Sim(cfg, st["radii"], st["x"], st["v"], st["w"])
    s3.set_state(0, mid["x"], mid["v"], mid["w"], F=mid["F"], T=mid["T"], s_le=mid["s_le"], step=mid["step"],
                 contacts=(ij, cs))
    s3.step(20)
    a, b, c = s1.get_state(), s2.get_state(), s3.get_state()
    for key in ("x", "v", "w", "F", "T"):
        assert np.array_equal(a[key], b[key]), key
        assert np.array_equal(a[key], c[key]), key


def test_health_errors(P):
    st = _state(n=300, phi=0.5)
    x = st["x"].copy()
    x[1] = (x[0] + np.array([0.5, 0.0, 0.0])) % st["L"][0]   # deep overlap
    _say("case: deep overlap rejected at creation")
    with pytest.raises(P.SimError) as e:
        P.Sim(_cfg(P, st), st["radii"], x, st["v"], st["w"])
    assert e.value.code == -4
    _say("case: more than 64 partners within the list range (skin 5) rejected")
    with pytest.raises(P.SimError) as e:
        P.Sim(_cfg(P, st, skin=5.0), st["radii"], st["x"], st["v"], st["w"])
    assert e.value.code == -5 and "at most 64" in str(e.value)
    # inputs the host rejects before anything reaches the GPU
    bad = [("NaN coordinate", "x", (3, 1), np.nan), ("coordinate equal to L", "x", (4, 2), st["L"][2]),
           ("infinite velocity", "v", (5, 0), np.inf), ("NaN angular velocity", "w", (6, 1), np.nan)]
    for what, key, (i, d), val in bad:
        _say(f"case: {what} rejected at creation")
        arr = {k: st[k].copy() for k in ("x", "v", "w")}
        arr[key][i, d] = val
        with pytest.raises(P.SimError) as e:
            P.Sim(_cfg(P, st), st["radii"], arr["x"], arr["v"], arr["w"])
        assert e.value.code == -1  # SIM_EINVAL
    sim = P.Sim(_cfg(P, st), st["radii"], st["x"], st["v"], st["w"])
    zero = np.zeros_like(st["x"])
    for what, F, T in (("NaN force", np.where(np.arange(3) == 1, np.nan, zero), zero),
                       ("infinite torque", zero, np.where(np.arange(3) == 2, np.inf, zero))):
        _say(f"case: {what} rejected by set_state")
        with pytest.raises(P.SimError) as e:
            sim.set_state(0, st["x"], st["v"], st["w"], F=F, T=T)
        assert e.value.code == -1  # SIM_EINVAL
    # contact tables the host rejects (partner id out of range, higher id first, more than 16 contacts
    # on one particle): nothing is uploaded, so the handle steps exactly as an untouched one
    n = len(st["radii"])
    moved = {k: st[k] + 0.0 for k in ("v", "w")}
    moved["v"][:, 0] += 0.25
    for what, cij in (("partner id out of range", np.array([[0, n]], np.uint32)),
                      ("higher id first", np.array([[5, 2]], np.uint32)),
                      ("17 contacts on one particle", np.array([[0, j] for j in range(1, 18)], np.uint32))):
        _say(f"case: contact table with {what} rejected by set_state")
        with pytest.raises(P.SimError) as e:
            sim.set_state(0, st["x"] * 0.5, moved["v"], moved["w"], contacts=(cij, np.zeros((len(cij), 3))))
        assert e.value.code == -1  # SIM_EINVAL
    ref = P.Sim(_cfg(P, st), st["radii"], st["x"], st["v"], st["w"])
    sim.step(20)
    ref.step(20)
    a, b = sim.get_state(), ref.get_state()
    for key in ("x", "v", "w", "F", "T"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(sim.stress_series(), ref.stress_series())
    sim.close()
    ref.close()


def test_large_sampled_fp64(P):
    """50,000 spheres at phi = 0.55: forces on sampled particles against the oracle one by one."""
    w = gen.C2
    st = gen.make_state(w)
    _say("case: N=50000 phi=0.55 FP64 sampled")
    sim = P.Sim(_cfg(P, st), st["radii"], st["x"], st["v"], st["w"])
    orc = O.Oracle(O.Params(L=st["L"], **st["params"], flags=O.CELLS), st["radii"], st["x"], st["v"], st["w"])
    _compare_eval(P, sim, orc, TOL_F64)
    # the one-by-one oracle used for spot checks of larger systems, on the same input
    Fg, Tg = sim.forces()
    zero = np.zeros((w.n, 3))
    one = O.Oracle(O.Params(L=st["L"], **st["params"]), st["radii"], st["x"], st["v"], st["w"], F=zero, T=zero)
    rng = np.random.default_rng(0)
    worst = 0.0
    for i in rng.choice(w.n, 40, replace=False):
        F, T, fa, ta = one.particle_force(int(i))
        worst = max(worst, np.linalg.norm(Fg[i] - F) / fa, np.linalg.norm(Tg[i] - T) / max(ta, 1e-300))
    _say(f"  worst sampled error {worst:.2e}")
    assert worst <= TOL_F64


def test_repulsion_matches_oracle(P):
    """Short-ranged repulsion (Sec. IV.F), A = 100 kT, on every pair with gap up to 16 kappa
    (beyond the lubrication cut-off too): forces, exact springs and the contact stress (which
    holds the repulsion) against the oracle, both precisions, and three steps."""
    st = _state(n=500, phi=0.5, seed=12)
    A = 100.0 * st["params"]["kT"]
    # the packing has pairs past the lubrication cut-off within the repulsion's range
    d = st["x"][:, None, :] - st["x"][None, :, :]
    d -= np.asarray(st["L"]) * np.rint(d / np.asarray(st["L"]))
    r = np.linalg.norm(d, axis=2)
    sa = st["radii"][:, None] + st["radii"][None, :]
    band = (r > 1.025 * sa) & (r <= 1.16 * sa)
    assert band.sum() // 2 > 100
    for prec, tol, exact in ((P.FP64, TOL_F64, True), (P.MIXED, TOL_MIX, False)):
        for lanes in (1, 2):
            _say(f"case: repulsion A=100 kT precision={prec} lanes={lanes}")
            sim = P.Sim(_cfg(P, st, precision=prec, repulsion=A, pair_kernel=3, lanes=lanes), st["radii"],
                        st["x"], st["v"], st["w"])
            orc = O.Oracle(O.Params(L=st["L"], rep_A=A, **st["params"]), st["radii"], st["x"], st["v"], st["w"])
            _compare_eval(P, sim, orc, tol, exact=exact)
    sim = P.Sim(_cfg(P, st, repulsion=A), st["radii"], st["x"], st["v"], st["w"])
    orc = O.Oracle(O.Params(L=st["L"], rep_A=A, **st["params"]), st["radii"], st["x"], st["v"], st["w"])
    sim.step(3)
    orc.step(3)
    gs, os_ = sim.get_state(), orc.state()
    assert np.abs(gs["x"] - os_["x"]).max() < 1e-11


def test_structural_stress_matches_oracle(P):
    """Structural Brownian stress (Sec. II.D) of the GPU state against the oracle's brute force,
    at creation and after 40 sheared steps (Lees-Edwards offset non-zero)."""
    st = _state(n=800, phi=0.55, seed=13)
    sim = P.Sim(_cfg(P, st, lanes=1), st["radii"], st["x"], st["v"], st["w"])
    for k in range(2):
        gs = sim.get_state()
        _say(f"case: structural stress N=800 after {40 * k} steps, s_le={gs['s_le']:.3e}")
        orc = O.Oracle(O.Params(L=st["L"], **st["params"]), st["radii"], gs["x"], gs["v"], gs["w"], s_le=gs["s_le"])
        Sg, So = sim.structural_stress(), orc.structural_stress()
        _say(f"  max rel err {np.abs(Sg - So).max() / np.abs(So).max():.2e}")
        assert np.abs(Sg - So).max() <= 1e-12 * np.abs(So).max()
        sim.step(40)
    # the rebuild it performs changes no trajectory: compare with a run that never asked
    ref = P.Sim(_cfg(P, st, lanes=1), st["radii"], st["x"], st["v"], st["w"])
    ref.step(80)
    a, b = sim.get_state(), ref.get_state()
    for key in ("x", "v", "w", "F", "T"):
        assert np.array_equal(a[key], b[key]), key


def test_rotational_couplings_match_oracle(P):
    """Rotational lubrication couplings and pairwise Brownian torques (SIM_LUB_ROT): forces,
    torques, exact springs and stresses against the oracle in both precisions and for 1 and 2
    cull lanes; with the repulsion as well; then a short FP64 trajectory."""
    st = _state(n=500, phi=0.5, seed=14)
    A = 10.0 * st["params"]["kT"]
    for prec, tol, exact in ((P.FP64, TOL_F64, True), (P.MIXED, TOL_MIX, False)):
        for lanes, rep in ((1, 0.0), (2, 0.0), (1, A)):
            _say(f"case: LUB_ROT precision={prec} lanes={lanes} repulsion={rep}")
            sim = P.Sim(_cfg(P, st, precision=prec, flags=P.LUB_ROT, pair_kernel=3, lanes=lanes, repulsion=rep),
                        st["radii"], st["x"], st["v"], st["w"])
            orc = O.Oracle(O.Params(L=st["L"], flags=O.LUB_ROT, rep_A=rep, **st["params"]), st["radii"], st["x"],
                           st["v"], st["w"])
            _compare_eval(P, sim, orc, tol, exact=exact)
    sim = P.Sim(_cfg(P, st, flags=P.LUB_ROT, repulsion=A), st["radii"], st["x"], st["v"], st["w"])
    orc = O.Oracle(O.Params(L=st["L"], flags=O.LUB_ROT, rep_A=A, **st["params"]), st["radii"], st["x"], st["v"],
                   st["w"])
    for k in range(3):
        sim.step(2)
        orc.step(2)
        gs, os_ = sim.get_state(), orc.state()
        dx = np.abs(gs["x"] - os_["x"]).max()
        dw = np.abs(gs["w"] - os_["w"]).max() / np.abs(os_["w"]).max()
        _say(f"  after {2 * (k + 1)} steps: |dx| {dx:.2e} |dw|/|w| {dw:.2e}")
        assert dx < 1e-11 and dw < 1e-9
        assert np.array_equal(sim.contacts()[0], orc.contacts()[0])


def test_displacement_msd_rdf_match_oracle(P):
    """Accumulated non-affine displacement and its mean square, and the pair-distance histogram of
    the sheared state, against the oracle (histogram bit-exact on the GPU's own state)."""
    st = _state(n=600, phi=0.5, seed=15)
    untracked = P.Sim(_cfg(P, st), st["radii"], st["x"], st["v"], st["w"])
    for call in (untracked.displacement, untracked.msd, untracked.reset_displacement):
        with pytest.raises(P.SimError) as e:   # kept only when asked for at creation
            call()
        assert e.value.code == -1
    sim = P.Sim(_cfg(P, st, flags=P.TRACK_DISPLACEMENT), st["radii"], st["x"], st["v"], st["w"])
    orc = O.Oracle(O.Params(L=st["L"], **st["params"]), st["radii"], st["x"], st["v"], st["w"])
    _say("case: displacement, MSD and g(r) after 40 sheared steps, N=600")
    untracked.step(40)
    sim.step(40)
    orc.step(40)
    dg, do = sim.displacement(), orc.displacement()
    err = np.abs(dg - do).max() / np.abs(do).max()
    _say(f"  displacement rel err {err:.2e}")
    assert err < 1e-10
    assert np.allclose(sim.msd(), (do ** 2).mean(axis=0), rtol=1e-9, atol=0)
    gs = sim.get_state()
    ref = O.Oracle(O.Params(L=st["L"], **st["params"]), st["radii"], gs["x"], gs["v"], gs["w"], s_le=gs["s_le"])
    r_max = 2.0 * 1.0 * 1.025 + 0.2
    hg, ho = sim.rdf(r_max, 50), ref.rdf(r_max, 50)
    _say(f"  g(r) pairs {hg.sum()} / {ho.sum()}")
    assert np.array_equal(hg, ho)
    # the tracking changes no trajectory
    gu = untracked.get_state()
    for key in ("x", "v", "w", "F", "T"):
        assert np.array_equal(gs[key], gu[key]), key
    untracked.close()
    sim.reset_displacement()
    assert np.abs(sim.displacement()).max() == 0.0
    with pytest.raises(P.SimError):
        sim.rdf(0.5 * st["L"][0], 50)   # not below half the box side: the minimum image would not be unique


def test_rdf_beyond_list_range_and_xy_slice(P):
    """g(r) counts out to 3 diameters (past the first shells, where the potential of mean force
    is flat) and the slice through the flow-gradient plane, from the library's own cell pass
    on a sheared state (Lees-Edwards offset non-zero), bit-exact against the oracle's brute
    force over all pairs of the same state."""
    st = _state(n=900, phi=0.5, pe=10.0, kT=None, seed=35)
    sim = P.Sim(_cfg(P, st), st["radii"], st["x"], st["v"], st["w"])
    sim.step(300)
    gs = sim.get_state()
    assert gs["s_le"] > 0.0
    ref = O.Oracle(O.Params(L=st["L"], **st["params"]), st["radii"], gs["x"], gs["v"], gs["w"], s_le=gs["s_le"])
    L = st["L"][0]
    for r_max, nb in ((6.0, 120), (0.49 * L, 64)):
        _say(f"case: g(r) counts to r_max={r_max:.3f}, N=900, s_le={gs['s_le']:.3e}")
        hg, ho = sim.rdf(r_max, nb), ref.rdf(r_max, nb)
        assert hg.sum() > 1000 and np.array_equal(hg, ho)
    for r_max, slab, nb in ((4.0, 1.0, 40), (5.0, 2.8, 25)):
        _say(f"case: xy slice r_max={r_max} slab={slab} bins={nb}")
        hg, ho = sim.rdf_xy(r_max, slab, nb), ref.rdf_xy(r_max, slab, nb)
        assert hg.sum() > 1000 and np.array_equal(hg, ho)
        assert np.array_equal(hg, hg[::-1, ::-1])   # each pair at r and -r
    with pytest.raises(P.SimError):
        sim.rdf_xy(0.5 * L / math.sqrt(2.0) + 0.01, 1.0, 10)   # its reach would exceed half the box


def test_stress_acf_stream_unbounded_matches_oracle(P):
    """The streaming autocorrelation over 12,000 recorded steps (past the 8,192-record ring) of
    the Brownian and the lubrication shear stress equals, bit for bit, the oracle's
    autocorrelation of the same series (read in chunks before the ring wraps)."""
    st = _state(n=300, phi=0.5, seed=36)
    sim = P.Sim(_cfg(P, st), st["radii"], st["x"], st["v"], st["w"])
    sim.step(10)
    for comp in (P.STRESS_BROWN, P.STRESS_LUB):
        _say(f"case: streaming autocorrelation of component {comp}, 12000 steps, 200 lags")
        sim.stress_acf_stream(comp, 0, 1, 200)
        sim.reset_stress()
        sim.stress_series()
        chunks = []
        for _ in range(4):
            sim.step(3000)
            chunks.append(sim.stress_series())
        s = np.concatenate(chunks)[:, comp, 0, 1]
        assert len(s) == 12000
        got = sim.stress_acf(comp, 0, 1, 200)
        assert np.array_equal(got, O.acf(s, 200))
        with pytest.raises(P.SimError):
            sim.stress_acf(comp, 0, 1, 20000)   # more lags than the ring or the stream holds
    sim.stress_acf_stream(0, 0, 0, 0)


def test_stress_acf_matches_series(P):
    st = _state(n=500, phi=0.5, seed=16)
    sim = P.Sim(_cfg(P, st), st["radii"], st["x"], st["v"], st["w"])
    sim.step(10)
    sim.reset_stress()
    sim.stress_series()
    sim.step(300)
    _say("case: stress autocorrelation over 300 records")
    series = sim.stress_series()   # reading the series does not consume the records the ACF uses
    assert len(series) == 300
    for comp in (P.STRESS_BROWN, P.STRESS_LUB):
        acf = sim.stress_acf(comp, 0, 1, 40)
        s = series[:, comp, 0, 1]
        ref = np.array([np.mean(s[: len(s) - k] * s[k:]) for k in range(40)])
        assert np.allclose(acf, ref, rtol=1e-12, atol=1e-30 * abs(ref[0]))


def test_dilute_msd_closed_form_gpu(P):
    """phi = 0.001: the one-body drag and noise alone give the Ornstein-Uhlenbeck MSD
    2 kT m / gamma^2 (gamma t / m - 1 + exp(-gamma t / m)) per axis (Sec. III.B)."""
    n, a, rho, eta, kT = 3000, 1.0, 0.1, 0.1, 1.0
    radii = np.full(n, a)
    Lb = (n * 4.0 / 3.0 * math.pi / 0.001) ** (1.0 / 3.0)
    rng = np.random.default_rng(17)
    x = gen.relaxed_positions(radii, Lb, 17)   # no overlaps
    m = 4.0 / 3.0 * math.pi * rho * a ** 3
    v = rng.standard_normal((n, 3)) * math.sqrt(kT / m)
    w = rng.standard_normal((n, 3)) * math.sqrt(kT / (0.4 * m * a * a))
    cfg = P.Config(box=(Lb, Lb, Lb), rho=rho, eta=eta, kT=kT, gammadot=0.0, dt=1e-4, seed=5,
                   flags=P.TRACK_DISPLACEMENT)
    sim = P.Sim(cfg, radii, x, v, w)
    gamma = 6 * math.pi * eta * a
    _say("case: dilute MSD, N=3000 phi=0.001")
    done = 0
    for steps in (500, 1500, 4000):
        sim.step(steps - done)
        done = steps
        t = steps * 1e-4
        expect = 2 * kT * m / gamma ** 2 * (gamma * t / m - 1 + math.exp(-gamma * t / m))
        msd = sim.msd()
        _say(f"  t={t:.2f}: MSD per axis {msd} expected {expect:.4e}")
        # each axis is a mean over 3000 independent particles: relative s.e. ~ sqrt(2/3000)
        assert np.all(np.abs(msd / expect - 1) < 6 * math.sqrt(2.0 / n))


@pytest.mark.parametrize("name, n, phi, radii_kind, mu, prec", [
    ("bidisperse N=1000000 phi=0.56", 1_000_000, 0.56, "bidisperse", 0.5, "mixed"),
    ("bidisperse N=1000000 phi=0.56 FP64", 1_000_000, 0.56, "bidisperse", 0.5, "fp64"),
    ("log-normal N=4000000 phi=0.58 mu=1", 4_000_000, 0.58, "lognormal", 1.0, "mixed"),
])
def test_full_size_sampled(P, name, n, phi, radii_kind, mu, prec):
    """The benchmark's launch configuration (half-pair kernel, one cull lane) at the full sizes
    of the 1M- and 4M-sphere workloads: forces and torques of sampled particles against the
    oracle's one-particle evaluation.  Positions are uniform random (overlaps allowed, the
    overlap limit raised), so no packing is needed; only the force law is compared."""
    rng = np.random.default_rng(n + 1)
    a = gen.radii_bidisperse(n, 3) if radii_kind == "bidisperse" else gen.radii_lognormal(n, 3)
    L = gen.box_length(a, phi)
    x = rng.random((n, 3)) * L
    gd, kT = gen.pe_to_rates(10.0)
    m = 4.0 / 3.0 * math.pi * 0.1 * a ** 3
    v = rng.standard_normal((n, 3)) * np.sqrt(kT / m)[:, None]
    v[:, 0] += gd * (x[:, 1] - 0.5 * L)
    w = rng.standard_normal((n, 3)) * np.sqrt(kT / (0.4 * m * a * a))[:, None]
    prm = dict(rho=0.1, eta=0.1, kn=1e4, kt=2e4 / 7, mu=mu, kT=kT, gammadot=gd, dt=1e-4, xi_cut=0.05,
               xi_min=1e-3, seed=7)
    _say(f"case: {name}, sampled forces at creation")
    cfg = P.Config(box=(L, L, L), precision=P.MIXED if prec == "mixed" else P.FP64, pair_kernel=3, lanes=1,
                   max_overlap=10.0, nlist_cap=64, **prm)
    sim = P.Sim(cfg, a, x, v, w)
    Fg, Tg = sim.forces()
    zero = np.zeros((n, 3))
    one = O.Oracle(O.Params(L=(L, L, L), **prm), a, x, v, w, F=zero, T=zero)
    worst = 0.0
    for i in rng.choice(n, 24, replace=False):
        F, T, fa, ta = one.particle_force(int(i))
        worst = max(worst, np.linalg.norm(Fg[i] - F) / fa, np.linalg.norm(Tg[i] - T) / max(ta, 1e-300))
    _say(f"  worst sampled error {worst:.2e}")
    assert worst <= (TOL_MIX if prec == "mixed" else TOL_F64)


def _stress_all(P, sim, r=0):
    """(5, 3, 3) contact, lubrication, Brownian, drag, total of the last evaluation."""
    return np.stack([sim.stress(r, c, P.STRESS_LAST) for c in range(5)])


def test_drag_total_stress_and_eta_r_match_oracle(P):
    """The drag stresslet (Sec. II.B), the total stress (Sec. IV.D) and eta_r (Sec. II.E) of the
    library against the oracle's, FP64, at creation and after sheared steps; the running mean
    of the total over the steps against the mean of the oracle's per-step totals."""
    st = _state(n=800, phi=0.55, pe=10.0, kT=None, seed=31)
    p = st["params"]
    sim = P.Sim(_cfg(P, st), st["radii"], st["x"], st["v"], st["w"])
    orc = O.Oracle(O.Params(L=st["L"], **p), st["radii"], st["x"], st["v"], st["w"])
    sim.reset_stress()
    tot = []
    for k in range(3):
        Sg, So = _stress_all(P, sim), orc.stress_all()
        scale = np.abs(So).reshape(5, 9).max(axis=1)
        err = float((np.abs(Sg - So).reshape(5, 9).max(axis=1) / scale).max())
        eg = Sg[4][0, 1] / (p["eta"] * p["gammadot"])
        eo = orc.eta_r()
        _say(f"case: stresses after {20 * k} steps: max rel err {err:.2e}, eta_r GPU {eg:.12g} oracle {eo:.12g}")
        assert err < TOL_F64
        assert abs(eg - eo) <= TOL_F64 * abs(eo)
        assert Sg[3][0, 1] == pytest.approx(2.5 * st["phi"] * p["eta"] * p["gammadot"], rel=1e-12)
        sim.step(20)
        ser = orc.step(20, series=True).reshape(20, 3, 3, 3)
        tot.append(ser[:, 0] + ser[:, 1])
    mean_o = np.concatenate(tot).mean(axis=0) + orc.stress_all()[3]
    mean_g = sim.stress(0, P.STRESS_TOTAL, P.STRESS_MEAN)
    assert np.abs(mean_g - mean_o).max() <= TOL_F64 * np.abs(mean_o).max()


def test_single_sphere_relaxes_to_imposed_flow_gpu(P):
    """One sphere at rest in shear flow, kT = 0: the library's one-body drag relaxes it towards
    U^inf = gammadot (y - Ly/2) e_x and Omega^inf = (0, 0, -gammadot/2) with the closed-form
    discrete law (1 - c)^2 (1 - 2c)^(n-1) of velocity-Verlet (c = zeta dt / 2m)."""
    L = (12.0, 10.0, 11.0)
    gd, eta, rho, dt, a = 0.7, 0.1, 0.1, 1e-4, 1.3
    y0 = 0.8 * L[1]
    x = np.array([[3.0, y0, 5.0]])
    v0 = np.array([[0.05, 0.0, -0.02]])
    w0 = np.array([[0.1, -0.3, 0.2]])
    for prec, tol in ((P.FP64, 1e-11), (P.MIXED, 1e-5)):
        _say(f"case: one sphere in shear, kT = 0, precision {prec}")
        sim = P.Sim(P.Config(box=L, gammadot=gd, kT=0.0, eta=eta, rho=rho, dt=dt, precision=prec), np.array([a]), x,
                    v0, w0)
        U = np.array([gd * (y0 - 0.5 * L[1]), 0.0, 0.0])
        Om = np.array([0.0, 0.0, -0.5 * gd])
        m = 4.0 / 3.0 * math.pi * rho * a ** 3
        I = 0.4 * m * a ** 2
        c = 6 * math.pi * eta * a * dt / (2 * m)
        cr = 8 * math.pi * eta * a ** 3 * dt / (2 * I)
        done = 0
        for nsteps in (1, 10, 300):
            sim.step(nsteps - done)
            done = nsteps
            g = sim.get_state()
            fac = (1 - c) ** 2 * (1 - 2 * c) ** (nsteps - 1)
            facr = (1 - cr) ** 2 * (1 - 2 * cr) ** (nsteps - 1)
            assert np.allclose(g["v"][0] - U, fac * (v0[0] - U), rtol=tol, atol=1e-17)
            assert np.allclose(g["w"][0] - Om, facr * (w0[0] - Om), rtol=tol, atol=1e-17)
        sim.close()


def test_positions_in_id_order_and_wrapped(P):
    """sim_positions returns the positions in id order, wrapped into [0, L), equal to the oracle's
    after sheared steps that carried particles across the Lees-Edwards boundary."""
    st = _state(n=700, phi=0.5, kT=1.0, seed=33)
    sim = P.Sim(_cfg(P, st), st["radii"], st["x"], st["v"], st["w"])
    orc = O.Oracle(O.Params(L=st["L"], **st["params"]), st["radii"], st["x"], st["v"], st["w"])
    _say("case: positions after 1000 steps, N=700, kT=1")
    sim.step(1000)
    orc.step(1000)
    xg, xo = sim.positions(), orc.state()["x"]
    assert xg.shape == (700, 3)
    assert np.all(xg >= 0.0) and np.all(xg < np.asarray(st["L"]))
    assert np.abs(xg - xo).max() < 1e-11
    assert np.array_equal(xg, sim.get_state()["x"])
    # particles near the top and bottom are carried by the flow across the x boundary (a jump of
    # almost L: each step moves them by far less)
    crossed = np.abs(xg[:, 0] - st["x"][:, 0]) > 0.5 * st["L"][0]
    _say(f"  {int(crossed.sum())} particles wrapped across x = L")
    assert crossed.any()


def test_torch_allocator(P):
    """A handle whose device memory comes from PyTorch's caching allocator (sim_set_allocator)
    steps bit-identically to one on hipMalloc, and frees into that allocator on destroy."""
    import torch
    st = _state(n=900, phi=0.55, seed=34)
    runs = []
    try:
        for use_torch in (False, True):
            if use_torch:
                P.use_torch_allocator()
                before = torch.cuda.memory_allocated()
            _say(f"case: 50 steps, device memory from torch: {use_torch}")
            sim = P.Sim(_cfg(P, st, lanes=1), st["radii"], st["x"], st["v"], st["w"])
            if use_torch:
                held = torch.cuda.memory_allocated() - before
                _say(f"  torch allocator holds {held} bytes for the handle")
                assert held > 1_000_000
            sim.step(50)
            runs.append(sim.get_state())
            sim.close()
            if use_torch:
                assert torch.cuda.memory_allocated() == before
    finally:
        P.use_default_allocator()
    for key in ("x", "v", "w", "F", "T"):
        assert np.array_equal(runs[0][key], runs[1][key]), key


def test_lists_regrow_to_partner_count(P):
    """A list capacity of 2 entries, far below the partner count: every build that finds
    more partners regrows the lists and builds them again, so the run is the run with
    room for 64 (same lists, same trajectory bit for bit), with a list build at every step."""
    st = _state(n=300, phi=0.5)
    _say("case: nlist_cap 2 vs 64, skin 3, 200 steps, a build per step")
    fl = P.REBUILD_EACH_STEP
    small = P.Sim(_cfg(P, st, flags=fl, nlist_cap=2, skin=3.0, lanes=1), st["radii"], st["x"], st["v"], st["w"])
    big = P.Sim(_cfg(P, st, flags=fl, nlist_cap=64, skin=3.0, lanes=1), st["radii"], st["x"], st["v"], st["w"])
    ls, lb = small.nlist(), big.nlist()
    cnt = np.bincount(ls.reshape(-1), minlength=300)
    _say(f"  list capacity {small.stats()['list_cap']} for at most {cnt.max()} partners")
    assert np.array_equal(ls, lb)
    assert cnt.max() <= small.stats()["list_cap"] <= 64 and small.stats()["list_cap"] > 2
    assert big.stats()["list_cap"] == 64
    small.step(200)
    big.step(200)
    a, b = small.get_state(), big.get_state()
    for key in ("x", "v", "w", "F", "T"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(small.nlist(), big.nlist())
    assert small.stats()["rebuilds"] == big.stats()["rebuilds"] >= 200
    small.close()
    big.close()


def test_kinetic_temperatures(P):
    """sim_stats' kinetic temperatures against the host's sums over the full-step
    velocities: sum m |v - U^inf(x)|^2 / 3n and sum I |w - Omega^inf|^2 / 3n with
    U^inf = gammadot (y - L_y/2) e_x and Omega^inf = -gammadot/2 e_z; after some steps of a
    Brownian run both are of order kT."""
    st = _state(n=500, phi=0.4, pe=1.0, kT=1.0)
    p = st["params"]
    for prec in (P.FP64, P.MIXED):
        sim = P.Sim(_cfg(P, st, precision=prec), st["radii"], st["x"], st["v"], st["w"])
        sim.step(400)
        g, stt = sim.get_state(), sim.stats()
        a = st["radii"]
        m = 4.0 / 3.0 * np.pi * p["rho"] * a ** 3
        inertia = 0.4 * m * a ** 2
        u = g["v"].copy()
        u[:, 0] -= p["gammadot"] * (g["x"][:, 1] - 0.5 * st["L"][1])
        om = g["w"].copy()
        om[:, 2] += 0.5 * p["gammadot"]
        kt = float((m * (u * u).sum(axis=1)).sum() / (3 * len(a)))
        kr = float((inertia * (om * om).sum(axis=1)).sum() / (3 * len(a)))
        _say(f"case: kinetic temperatures precision {prec}: translational {stt['kT_translational']:.6g} "
             f"(host {kt:.6g}) rotational {stt['kT_rotational']:.6g} (host {kr:.6g})")
        assert abs(stt["kT_translational"] - kt) <= 1e-12 * kt
        assert abs(stt["kT_rotational"] - kr) <= 1e-12 * kr
        assert 0.6 < kt < 1.6 and 0.6 < kr < 1.6
        sim.close()
