"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: published
known-answer vectors, textbook special cases, closed forms, invariants, brute
force over all periodic images, or exact discrete-time statistics.
"""
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from inputs import gen

HERE = os.path.dirname(os.path.abspath(__file__))
PI = math.pi


def _params(L, **kw):
    p = O.Params(L=tuple(L))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# --------------------------------------------------------------------------
# RNG: Philox4x32-10 and Box-Muller
# --------------------------------------------------------------------------
def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, out in _kat():
        assert list(O.philox4x32_10(ctr, key)) == out


def test_philox_matches_pytorch_header(tmp_path):
    """Cross-check against PyTorch's open-source Philox engine header (compiled here, host only)."""
    import torch.utils.cpp_extension as ce
    inc = ce.include_paths()[0]
    hdr = os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")
    if not os.path.exists(hdr):
        pytest.skip("PyTorch headers not installed")
    src = tmp_path / "p.cpp"
    src.write_text(r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  unsigned long long seed = strtoull(argv[1], 0, 0), sub = strtoull(argv[2], 0, 0), off = strtoull(argv[3], 0, 0);
  at::philox_engine e(seed, sub, off);
  for (int q = 0; q < 4; ++q) printf("%u ", e());
  printf("\n");
  return 0;
}
""")
    exe = tmp_path / "p"
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, str(src), "-o", str(exe)], capture_output=True)
    if r.returncode != 0:
        pytest.skip("could not compile the PyTorch header: " + r.stderr.decode()[-300:])
    rng = np.random.default_rng(5)
    for _ in range(20):
        seed, sub, off = (int(t) for t in rng.integers(0, 2 ** 63, size=3))
        outs = [int(t) for t in subprocess.check_output([str(exe), str(seed), str(sub), str(off)]).split()]
        ctr = [off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert list(O.philox4x32_10(ctr, key)) == outs


def test_box_muller_moments():
    from scipy import stats
    g = np.array([O.gauss3(12345, k, 7, 0xFFFFFFFF, 2) for k in range(60000)]).reshape(-1)
    assert abs(g.mean()) < 5 / math.sqrt(g.size)
    assert abs(g.var() - 1.0) < 5 * math.sqrt(2.0 / g.size)
    assert abs(stats.kurtosis(g, fisher=False) - 3.0) < 5 * math.sqrt(24.0 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-4


def test_noise_streams_uncorrelated():
    a = np.array([O.gauss3(9, k, 3, 0xFFFFFFFF, 2) for k in range(20000)])
    b = np.array([O.gauss3(9, k, 3, 0xFFFFFFFF, 3) for k in range(20000)])
    c = np.array([O.gauss3(9, k, 3, 5, 0) for k in range(20000)])
    for u, v in ((a, b), (a, c), (b, c)):
        cc = (u * v).mean(axis=0)
        assert np.all(np.abs(cc) < 5 / math.sqrt(len(u)))


# --------------------------------------------------------------------------
# Lubrication scalars X^A_11, Y^A_11 (Sec. II.B)
# --------------------------------------------------------------------------
def _golden_xa():
    rows = []
    for line in open(os.path.join(HERE, "golden", "lubrication_scalars.txt")):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([float(t) for t in line.split()])
    return rows


def test_lub_equal_spheres_textbook():
    """beta = 1: X^A/(6 pi eta a) = 1/(4 xi) + 9/40 ln(1/xi), Y^A/(6 pi eta a) = 1/6 ln(1/xi)."""
    for a in (0.6, 1.0, 1.4):
        for xi in (1e-3, 1e-2, 0.05):
            xa, ya = O.lub_scalars(0.1, a, a, xi)
            s = 6 * PI * 0.1 * a
            assert xa / s == pytest.approx(1 / (4 * xi) + 0.225 * math.log(1 / xi), rel=1e-14)
            assert ya / s == pytest.approx(math.log(1 / xi) / 6, rel=1e-14)


def test_lub_golden_values():
    for eta, ai, aj, xi, xa_ref, ya_ref in _golden_xa():
        xa, ya = O.lub_scalars(eta, ai, aj, xi)
        assert xa == pytest.approx(xa_ref, rel=2e-4)
        assert ya == pytest.approx(ya_ref, rel=2e-4)


def test_lub_symmetric_and_reynolds_limit():
    """X^A, Y^A are symmetric in (a_i, a_j); the 1/xi part is Reynolds' 6 pi eta a*^2 / h."""
    rng = np.random.default_rng(2)
    for _ in range(200):
        ai, aj = rng.uniform(0.6, 1.6, 2)
        xi = 10 ** rng.uniform(-3, math.log10(0.05))
        x1, y1 = O.lub_scalars(0.1, ai, aj, xi)
        x2, y2 = O.lub_scalars(0.1, aj, ai, xi)
        assert x1 == pytest.approx(x2, rel=1e-13)
        assert y1 == pytest.approx(y2, rel=1e-13)
    ai, aj = 0.8, 1.5
    astar = ai * aj / (ai + aj)
    # X^A(xi) = c1/xi + c2 ln(1/xi): remove the log part using two gaps
    xs = [1e-3, 2e-3]
    vals = [O.lub_scalars(0.1, ai, aj, xi)[0] for xi in xs]
    l1, l2 = (math.log(1 / x) for x in xs)
    # solve for c1, c2
    A = np.array([[1 / xs[0], l1], [1 / xs[1], l2]])
    c1, c2 = np.linalg.solve(A, vals)
    h_over_xi = (ai + aj) / 2  # h = xi (a_i + a_j) / 2
    # c1 / xi = c1 (h / xi) / h must equal 6 pi eta a*^2 / h
    assert c1 * h_over_xi == pytest.approx(6 * PI * 0.1 * astar ** 2, rel=1e-10)


# --------------------------------------------------------------------------
# Two-sphere force law: lubrication, contact, Brownian, stress
# --------------------------------------------------------------------------
HEAVY = 1e12   # density making masses so large that velocities stay put


def _two(gap_xi, a=(1.0, 1.0), v=((0, 0, 0), (0, 0, 0)), w=((0, 0, 0), (0, 0, 0)), direction=(1, 0, 0),
         flags=0, L=20.0, **kw):
    a = np.array(a, float)
    n = np.array(direction, float)
    n /= np.linalg.norm(n)
    sa = a.sum()
    dist = sa * (1 + gap_xi / 2)
    c = np.array([L / 2, L / 2, L / 2])
    # r = x_i - x_j = dist * n, particle 0 is i
    x = np.array([c + 0.5 * dist * n, c - 0.5 * dist * n])
    p = _params((L, L, L), flags=flags, **kw)
    return O.Oracle(p, a, x, np.array(v, float), np.array(w, float)), n, dist


def test_lubrication_two_spheres_closed_form():
    eta = 0.1
    for xi in (2e-3, 0.01, 0.04):
        U = np.array([0.3, -0.2, 0.5])
        o, n, dist = _two(xi, v=((0, 0, 0), U), flags=O.NO_PAIR_BROWN | O.NO_CONTACT | O.NO_ONEBODY, eta=eta)
        F = o.state()["F"]
        s = 6 * PI * eta * 1.0
        XA = s * (1 / (4 * xi) + 0.225 * math.log(1 / xi))
        YA = s * math.log(1 / xi) / 6
        un = U @ n
        expect = XA * un * n + YA * (U - un * n)
        assert np.allclose(F[0], expect, rtol=1e-12, atol=0)
        assert np.array_equal(F[1], -F[0])


def test_lubrication_resists_approach_and_projects():
    fl = O.NO_PAIR_BROWN | O.NO_CONTACT | O.NO_ONEBODY
    # i (particle 0) moves toward j: force on i must point away from j (along +n)
    o, n, _ = _two(0.01, v=(-0.1 * np.array([1, 0, 0]), (0, 0, 0)), flags=fl)
    F = o.state()["F"]
    assert F[0] @ n > 0 and np.allclose(F[0][1:], 0, atol=1e-15)
    # pure tangential relative motion gives no normal force
    o, n, _ = _two(0.01, v=((0, 0, 0), (0, 0.2, 0)), flags=fl)
    F = o.state()["F"]
    assert abs(F[0] @ n) < 1e-15 and F[0][1] > 0


def test_lubrication_regularisation_and_cutoff():
    fl = O.NO_PAIR_BROWN | O.NO_CONTACT | O.NO_ONEBODY
    U = ((0, 0, 0), (0.1, 0.1, 0.0))
    F_min = _two(1e-3, v=U, flags=fl)[0].state()["F"][0]
    for xi in (5e-4, 1e-5, -0.01):
        F = _two(xi, v=U, flags=fl)[0].state()["F"][0]
        assert np.allclose(F, F_min, rtol=1e-12)
    assert np.all(_two(0.0501, v=U, flags=fl)[0].state()["F"] == 0)
    assert np.any(_two(0.0499, v=U, flags=fl)[0].state()["F"] != 0)


def test_normal_contact_repulsive_hookean():
    kn = 1e4
    for delta in (1e-4, 1e-3):
        xi = -2 * delta / 2.0
        o, n, _ = _two(xi, flags=O.NO_PAIR_BROWN | O.NO_LUB | O.NO_ONEBODY, kn=kn)
        F = o.state()["F"]
        assert np.allclose(F[0], kn * delta * n, rtol=1e-9)
        assert np.array_equal(F[1], -F[0])


def test_tangential_spring_slip_closed_form():
    """Fixed overlap, constant sliding velocity v: |s| = v t until mu k_n delta / k_t, then constant."""
    kn, kt, mu, dt = 1e4, 2e4 / 7, 0.5, 1e-4
    delta = 1e-3
    vslide = 0.7
    fl = O.NO_PAIR_BROWN | O.NO_LUB | O.NO_ONEBODY | O.FREEZE_X
    o, n, _ = _two(-delta, v=((0, vslide, 0), (0, 0, 0)), flags=fl, kn=kn, kt=kt, mu=mu, dt=dt, rho=HEAVY)
    limit = mu * kn * delta / kt
    for k in range(1, 80):
        o.step(1)
        ij, s, sl = o.contacts()
        assert len(ij) == 1
        expect = min(vslide * dt * (k + 1), limit)   # the evaluation at creation already added one increment
        assert np.linalg.norm(s[0]) == pytest.approx(expect, rel=1e-9)
        assert bool(sl[0]) == (vslide * dt * (k + 1) > limit)
        F = o.state()["F"]
        Ft = F[0] - (F[0] @ n) * n
        assert np.linalg.norm(Ft) == pytest.approx(kt * expect, rel=1e-9)
        assert Ft[1] < 0  # opposes the sliding of i along +y
    # torques: T_i / a_i == T_j / a_j, equal to lever arm x tangential force
    T = o.state()["T"]
    assert np.allclose(T[0], T[1], rtol=1e-12)
    F = o.state()["F"]
    Ft = F[0] - (F[0] @ n) * n
    assert np.allclose(T[0], np.cross(-1.0 * n, Ft), rtol=1e-9)


def test_frictionless_and_rolling():
    fl = O.NO_PAIR_BROWN | O.NO_LUB | O.NO_ONEBODY | O.FREEZE_X
    o, n, _ = _two(-1e-3, v=((0, 0.5, 0), (0, 0, 0)), flags=fl, mu=0.0, rho=HEAVY)
    o.step(5)
    F = o.state()["F"]
    assert np.allclose(F[0] - (F[0] @ n) * n, 0, atol=1e-14)
    # gears: a_i w_i + a_j w_j = 0 gives zero contact-point slip, s stays zero
    a = (1.0, 1.4)
    om = np.array([0, 0, 2.0])
    o, n, _ = _two(-1e-3, a=a, w=(om, -a[0] / a[1] * om), flags=fl, rho=HEAVY)
    o.step(3)
    _, s, _ = o.contacts()
    assert np.allclose(s, 0, atol=1e-15)


def test_spring_rotates_with_pair():
    """A stored spring is carried into the new tangent plane with its length kept."""
    fl = O.NO_PAIR_BROWN | O.NO_LUB | O.NO_ONEBODY
    L = 20.0
    a = np.array([1.0, 1.0])
    th = 0.3
    n = np.array([math.cos(th), math.sin(th), 0.0])
    dist = 2.0 - 1e-3
    c = np.full(3, L / 2)
    x = np.array([c + 0.5 * dist * n, c - 0.5 * dist * n])
    s0 = np.array([[0.0, 2e-4, 1e-4]])  # tangent to the old normal (1,0,0)
    o = O.Oracle(_params((L, L, L), flags=fl), a, x, np.zeros((2, 3)), np.zeros((2, 3)),
                 contacts=(np.array([[0, 1]]), s0))
    _, s, _ = o.contacts()
    assert np.linalg.norm(s[0]) == pytest.approx(np.linalg.norm(s0[0]), rel=1e-12)
    assert abs(s[0] @ n) < 1e-18


def test_pair_brownian_covariance_fdt():
    """<F^B (x) F^B> = (2 kT / dt)(X^A N + Y^A T) for a frozen pair (Sec. II.C)."""
    kT, dt, eta = 0.7, 1e-3, 0.1
    xi = 0.01
    fl = O.NO_LUB | O.NO_CONTACT | O.NO_ONEBODY | O.FREEZE_X
    o, n, _ = _two(xi, a=(1.0, 1.4), direction=(1, 2, -1), flags=fl, kT=kT, dt=dt, eta=eta, rho=HEAVY, seed=77)
    ns = 40000
    Fs = np.empty((ns, 3))
    for t in range(ns):
        o.step(1)
        st = o.state()
        Fs[t] = st["F"][0]
        assert np.array_equal(st["F"][1], -st["F"][0])
    xa, ya = O.lub_scalars(eta, 1.0, 1.4, xi)
    N = np.outer(n, n)
    R = (2 * kT / dt) * (xa * N + ya * (np.eye(3) - N))
    cov = Fs.T @ Fs / ns
    # compare in the eigenbasis: normal variance and in-plane variances
    evn = n @ cov @ n
    assert evn == pytest.approx(n @ R @ n, rel=5 * math.sqrt(2 / ns))
    t1 = np.cross(n, [0, 0, 1.0]); t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    for t in (t1, t2):
        assert t @ cov @ t == pytest.approx(t @ R @ t, rel=5 * math.sqrt(2 / ns))
    scale = math.sqrt((n @ R @ n) * (t1 @ R @ t1))
    assert abs(n @ cov @ t1) < 5 * scale / math.sqrt(ns)
    # no correlation between successive steps
    lag = (Fs[1:] * Fs[:-1]).sum(axis=1).mean() / np.trace(R)
    assert abs(lag) < 5 * math.sqrt(3) / math.sqrt(ns)


def test_one_body_brownian_covariance():
    """<F F> = (2kT/dt) 6 pi eta a I and <T T> = (2kT/dt) 8 pi eta a^3 I (Sec. II.C)."""
    kT, dt, eta, a = 0.3, 1e-3, 0.1, 1.4
    fl = O.FREEZE_X
    L = 20.0
    o = O.Oracle(_params((L, L, L), flags=fl, kT=kT, dt=dt, eta=eta, rho=HEAVY, seed=3), np.array([a]),
                 np.array([[L / 2, L / 2, 3.0]]), np.zeros((1, 3)), np.zeros((1, 3)))
    ns = 40000
    F = np.empty((ns, 3)); T = np.empty((ns, 3))
    for t in range(ns):
        o.step(1)
        st = o.state()
        F[t] = st["F"][0]; T[t] = st["T"][0]
    cf = F.T @ F / ns
    ct = T.T @ T / ns
    tol = 5 * math.sqrt(2 / ns)
    assert np.allclose(np.diag(cf), (2 * kT / dt) * 6 * PI * eta * a, rtol=tol)
    assert np.allclose(np.diag(ct), (2 * kT / dt) * 8 * PI * eta * a ** 3, rtol=tol)
    assert np.all(np.abs(cf - np.diag(np.diag(cf))) < 5 * np.mean(np.diag(cf)) / math.sqrt(ns))


def test_single_pair_stress_closed_form_and_label_swap():
    L = 20.0
    rng = np.random.default_rng(4)
    for trial in range(5):
        x = np.array([[8.0, 9.0, 10.0], [8.0, 9.0, 10.0]])
        d = rng.normal(size=3); d /= np.linalg.norm(d)
        x[1] = x[0] - (2.4 - 3e-3) * d
        v = rng.normal(size=(2, 3)) * 0.1
        w = rng.normal(size=(2, 3)) * 0.1
        a = np.array([1.0, 1.4])
        o1 = O.Oracle(_params((L, L, L), seed=11, flags=O.NO_ONEBODY), a, x, v, w)
        o2 = O.Oracle(_params((L, L, L), seed=11, flags=O.NO_ONEBODY), a[::-1].copy(), x[::-1].copy(),
                      v[::-1].copy(), w[::-1].copy())
        S1 = o1.stress()
        S2 = o2.stress()
        F = o1.state()["F"]
        r = x[0] - x[1]
        V = L ** 3
        assert np.allclose(S1.sum(axis=0), -np.outer(F[0], r) / V, rtol=1e-12, atol=1e-18)
        # contact and lubrication parts are label independent (noise is keyed by ids, so skip it)
        assert np.allclose(S1[0], S2[0], rtol=1e-12, atol=1e-18)
        assert np.allclose(S1[1], S2[1], rtol=1e-12, atol=1e-18)


# --------------------------------------------------------------------------
# Geometry: sheared periodic images and the pair set
# --------------------------------------------------------------------------
def _brute_all_images(x, a, L, s, xi_cut):
    """Pairs whose nearest image among all 27 sheared images is within the cut-off."""
    n = len(a)
    out = set()
    for i in range(n):
        for j in range(i + 1, n):
            best = np.inf
            for kx in (-1, 0, 1):
                for ky in (-1, 0, 1):
                    for kz in (-1, 0, 1):
                        img = x[j] + np.array([kx * L[0] + ky * s, ky * L[1], kz * L[2]])
                        # also allow the x-shifted neighbours of a sheared row
                        for kk in (-1, 0, 1):
                            d = x[i] - (img + np.array([kk * L[0], 0, 0]))
                            best = min(best, float(np.sqrt(d @ d)))
            rc = (a[i] + a[j]) * (1 + 0.5 * xi_cut)
            out.add(((i, j), best - rc))
    return out


@pytest.mark.parametrize("s_frac", [0.0, 1.0 / 3.0, 1.0 - 1e-12])
def test_pair_set_matches_all_images_and_cells(s_frac):
    n = 150
    L = (9.0, 8.0, 10.0)
    rng = np.random.default_rng(int(s_frac * 1000) + 1)
    a = rng.choice([1.0, 1.4], size=n)
    x, v, w = gen.random_state(n, L, a, seed=3)
    s = s_frac * L[0]
    o = O.Oracle(_params(L), a, x, v, w, s_le=s)
    got = {tuple(p) for p in o.pairs()}
    ref = _brute_all_images(x, a, L, s, 0.05)
    for (ij, margin) in ref:
        if margin < -1e-9:
            assert ij in got
        elif margin > 1e-9:
            assert ij not in got
    oc = O.Oracle(_params(L, flags=O.CELLS), a, x, v, w, s_le=s)
    assert np.array_equal(oc.pairs(), o.pairs())


def test_cells_bit_exact_large():
    n = 2000
    L = (30.0, 30.0, 30.0)
    a = gen.radii_bidisperse(n, 1)
    x, v, w = gen.random_state(n, L, a, seed=5)
    for s in (0.0, 11.3, L[0] - 1e-9):
        o1 = O.Oracle(_params(L, seed=4), a, x, v, w, s_le=s)
        o2 = O.Oracle(_params(L, seed=4, flags=O.CELLS), a, x, v, w, s_le=s)
        assert np.array_equal(o1.pairs(), o2.pairs())
        c1 = o1.contacts(); c2 = o2.contacts()
        assert np.array_equal(c1[0], c2[0]) and np.array_equal(c1[1], c2[1])
        assert np.allclose(o1.state()["F"], o2.state()["F"], rtol=1e-12, atol=1e-9)


def test_lees_edwards_offset_equivalent_to_flipped_tilt():
    """Offsets s and s - Lx describe the same image lattice (the remap at strain 0.5 -> -0.5)."""
    n = 300
    L = (12.0, 12.0, 12.0)
    a = gen.radii_bidisperse(n, 2)
    x, v, w = gen.random_state(n, L, a, seed=9)
    s = 0.7 * L[0]
    o1 = O.Oracle(_params(L, seed=2, flags=O.NO_PAIR_BROWN), a, x, v, w, s_le=s)
    o2 = O.Oracle(_params(L, seed=2, flags=O.NO_PAIR_BROWN), a, x, v, w, s_le=s - L[0])
    assert np.array_equal(o1.pairs(), o2.pairs())
    assert np.allclose(o1.state()["F"], o2.state()["F"], rtol=1e-10, atol=1e-9)


def test_boundary_crossing_keeps_peculiar_velocity():
    L = 10.0
    gd = 0.5
    x = np.array([[5.0, L - 1e-6, 5.0]])
    v = np.array([[gd * (L - 1e-6 - L / 2) + 0.01, 0.3, 0.0]])
    p = _params((L, L, L), gammadot=gd, flags=O.NO_ONEBODY, dt=1e-4)
    o = O.Oracle(p, np.array([1.0]), x, v, np.zeros((1, 3)))
    o.step(1)
    st = o.state()
    assert st["x"][0, 1] < 1.0  # re-entered at the bottom
    pec = st["v"][0, 0] - gd * (st["x"][0, 1] - L / 2)
    assert pec == pytest.approx(0.01, abs=1e-3)


# --------------------------------------------------------------------------
# Conservation and exact discrete-time statistics
# --------------------------------------------------------------------------
def test_pair_forces_conserve_momentum():
    n = 400
    w_ = gen.Workload("t", n, 0.5, 1.0, kT=1.0)
    st = gen.make_state(w_)
    p = O.Params(L=st["L"], **st["params"], flags=O.NO_ONEBODY)
    o = O.Oracle(p, st["radii"], st["x"], st["v"], st["w"])
    o.step(20)
    F = o.state()["F"]
    Fa, _ = o.norms()
    assert np.all(np.abs(F.sum(axis=0)) <= 1e-13 * Fa.sum())


def test_equipartition_exact_discrete():
    """Frozen positions, no shear: with forces evaluated at half-step velocities the
    full-step velocities have covariance exactly kT/m per component, for any stable
    damping, lubrication pairs included (the lubrication and its noise obey FDT)."""
    kT, dt, rho = 0.5, 0.1, 1.0
    L = 12.0
    # a small cluster with lubrication gaps (xi ~ 0.04) but no contacts; dt is
    # chosen so that the explicit lubrication damping stays stable
    x = np.array([[4.0, 4.0, 4.0], [6.04, 4.0, 4.0], [4.0, 6.045, 4.0], [6.045, 6.045, 4.0],
                  [8.0, 8.0, 8.0], [10.448, 8.0, 8.0]])
    a = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.4])
    m = 4 / 3 * PI * rho * a ** 3
    inertia = 0.4 * m * a ** 2
    p = _params((L, L, L), kT=kT, dt=dt, rho=rho, flags=O.FREEZE_X, seed=21)
    o = O.Oracle(p, a, x, np.zeros((6, 3)), np.zeros((6, 3)))
    assert len(o.pairs()) >= 4 and len(o.contacts()[0]) == 0
    o.step(2000)
    ns = 60000
    ev = np.zeros(6); ew = np.zeros(6)
    for t in range(ns // 200):
        o.step(200)
        st = o.state()
        ev += (m[:, None] * st["v"] ** 2).sum(axis=1) / 3
        ew += (inertia[:, None] * st["w"] ** 2).sum(axis=1) / 3
    ev /= ns // 200; ew /= ns // 200
    # 300 samples x 3 components, decorrelated by 200 steps
    tol = 5 * math.sqrt(2.0 / (3 * (ns // 200)))
    assert np.allclose(ev / kT, 1.0, atol=tol)
    assert np.allclose(ew / kT, 1.0, atol=tol)


def test_dilute_msd_closed_form():
    """Isolated spheres: <x^2> = 2 kT m / gamma^2 (gamma t / m - 1 + exp(-gamma t / m)) (Sec. III.B)."""
    n = 64
    L = 400.0
    kT, dt, rho, eta, a = 1.0, 5e-4, 0.1, 0.1, 1.0
    rng = np.random.default_rng(8)
    x = rng.random((n, 3)) * L
    m = 4 / 3 * PI * rho * a ** 3
    g = 6 * PI * eta * a
    v = rng.standard_normal((n, 3)) * math.sqrt(kT / m)
    p = _params((L, L, L), kT=kT, dt=dt, rho=rho, eta=eta, seed=5)
    o = O.Oracle(p, np.full(n, a), x, v, np.zeros((n, 3)))
    x0 = o.state()["x"].copy()
    disp = np.zeros((n, 3))
    prev = x0.copy()
    checkpoints = {200: None, 800: None, 3000: None}
    t = 0
    for stop in sorted(checkpoints):
        while t < stop:
            o.step(50)
            t += 50
            cur = o.state()["x"]
            d = cur - prev
            d -= L * np.rint(d / L)
            disp += d
            prev = cur.copy()
        checkpoints[stop] = (disp ** 2).mean()
    for stop, msd in checkpoints.items():
        tt = stop * dt
        ref = 2 * kT * m / g ** 2 * (g * tt / m - 1 + math.exp(-g * tt / m))
        # 192 independent components: relative sd sqrt(2/192)
        assert msd == pytest.approx(ref, rel=5 * math.sqrt(2 / (3 * n)))


def test_msd_two_printed_forms_agree():
    """The dimensional and the timescale forms of the MSD in Sec. III.B are the same function."""
    rho, eta, a, kT = 0.1, 0.1, 1.0, 0.017
    m = 4 / 3 * PI * rho * a ** 3
    g = 6 * PI * eta * a
    tI = rho * a ** 2 / eta
    tB = eta * a ** 3 / kT
    for t in (0.01, 0.3, 5.0):
        f1 = 2 * kT * m / g ** 2 * (g * t / m - 1 + math.exp(-g * t / m))
        f2 = a ** 2 * 2 / (27 * PI) * tI / tB * (4.5 * t / tI - 1 + math.exp(-4.5 * t / tI))
        assert f1 == pytest.approx(f2, rel=1e-12)


def test_sheared_contact_network_positive_viscosity():
    """Under shear the contact + lubrication shear stress is positive (eta_r > 0)."""
    w_ = gen.Workload("t", 300, 0.55, 100.0, steps=0)
    st = gen.make_state(w_)
    prm = dict(st["params"])
    prm["gammadot"] = 0.5
    p = O.Params(L=st["L"], **prm, flags=O.CELLS)
    o = O.Oracle(p, st["radii"], st["x"], st["v"], st["w"])
    ser = o.step(400, series=True).reshape(-1, 3, 3, 3)
    sxy = ser[100:, 0, 0, 1] + ser[100:, 1, 0, 1]
    assert sxy.mean() > 0


def test_restart_bit_exact():
    w_ = gen.Workload("t", 200, 0.5, 1.0, kT=1.0)
    st = gen.make_state(w_)
    p = O.Params(L=st["L"], **st["params"])
    o = O.Oracle(p, st["radii"], st["x"], st["v"], st["w"])
    o.step(30)
    mid = o.state()
    ij, s, _ = o.contacts()
    o.step(30)
    end = o.state()
    o2 = O.Oracle(p, st["radii"], mid["x"], mid["v"], mid["w"], s_le=mid["s_le"], step=mid["step"],
                  contacts=(ij, s), F=mid["F"], T=mid["T"])
    o2.step(30)
    end2 = o2.state()
    for k in ("x", "v", "w", "F", "T"):
        assert np.array_equal(end[k], end2[k])


def test_table1_peclet_numbers():
    """Sec. II.F: Pe = 6 pi eta a^3 gammadot / kT reproduces Table 1 to its printed precision."""
    for line in open(os.path.join(HERE, "golden", "table1_parameters.txt")):
        if line.startswith("#") or not line.strip():
            continue
        pe, gd, kT, a, rho, kn, eta = (float(t) for t in line.split())
        assert 6 * PI * eta * a ** 3 * gd / kT == pytest.approx(pe, rel=0.05)
        g2, k2 = gen.pe_to_rates(pe, eta)
        assert 6 * PI * eta * g2 / k2 == pytest.approx(pe, rel=1e-12)


# --------------------------------------------------------------------------
# Short-ranged repulsion (Sec. IV.F) and the structural Brownian stress (Sec. II.D)
# --------------------------------------------------------------------------
ONLY_REP = O.NO_LUB | O.NO_PAIR_BROWN | O.NO_CONTACT | O.NO_ONEBODY


def test_repulsion_two_spheres_closed_form():
    A = 0.7
    for a in ((1.0, 1.0), (1.0, 1.4)):
        for xi in (-4e-3, 0.0, 0.01, 0.049, 0.06, 0.2, 0.3199):
            o, n, dist = _two(xi, a=a, flags=ONLY_REP | O.FREEZE_X, rep_A=A, direction=(0.3, -0.5, 0.8))
            F = o.state()["F"]
            sa = sum(a)
            kappa = 0.01 * sa
            expect = A / kappa * math.exp(-(dist - sa) / kappa) * n   # pushes particle 0 away from 1
            assert np.allclose(F[0], expect, rtol=1e-12, atol=0), (a, xi)
            assert np.array_equal(F[1], -F[0])
            assert np.abs(o.state()["T"]).max() == 0.0
            # kept with the contact stress: -F (x) r / V, r = x_0 - x_1
            S = o.stress()
            V = 20.0 ** 3
            assert np.allclose(S[0], -np.outer(F[0], dist * n) / V, rtol=1e-12, atol=1e-30)
            assert np.abs(S[1]).max() == 0.0 and np.abs(S[2]).max() == 0.0


def test_repulsion_range_and_adds_to_contact():
    """The repulsion acts up to a gap of 16 kappa = 0.16 (a_i + a_j) (xi = 0.32), where it has
    decayed to exp(-16) of its contact value, beyond the lubrication cut-off; those pairs are
    not lubrication pairs (no interaction-set entry, no pair noise)."""
    o, n, dist = _two(0.3201, flags=ONLY_REP, rep_A=1.0)
    assert np.abs(o.state()["F"]).max() == 0.0
    o, n, dist = _two(0.3199, flags=O.NO_CONTACT | O.NO_ONEBODY, rep_A=1.0, kT=1.0)
    F = o.state()["F"][0]
    assert len(o.pairs()) == 0
    assert np.allclose(F, 1.0 / 0.02 * math.exp(-(dist - 2.0) / 0.02) * n, rtol=1e-12, atol=0)
    assert F @ n / (1.0 / 0.02) < 1.2e-7
    # with contact on: Hookean part plus the repulsion, both along n
    kn = 1e4
    o, n, dist = _two(-2e-3, flags=O.NO_LUB | O.NO_PAIR_BROWN | O.NO_ONEBODY, rep_A=0.5, kn=kn, mu=0.0)
    F = o.state()["F"][0]
    delta = 2.0 - dist
    expect = (kn * delta + 0.5 / 0.02 * math.exp(delta / 0.02)) * n
    assert np.allclose(F, expect, rtol=1e-12, atol=0)


def test_structural_stress_shells():
    """Bidisperse pair: the shell of each particle is 0.05 a_i, so a gap between 0.05 and 0.07
    counts only on the larger sphere's side; the tensor is -(kT/V) sum (a_i/Delta_i) n n."""
    L, kT = 20.0, 0.3
    u = np.array([1.0, 2.0, -2.0]) / 3.0
    for h, weight in ((0.03, 40.0), (0.06, 20.0), (0.08, 0.0), (-0.01, 40.0)):
        c = np.array([10.0, 10.0, 10.0])
        x = np.array([c, c - (2.4 + h) * u])
        o = O.Oracle(_params((L, L, L), kT=kT), np.array([1.0, 1.4]), x, np.zeros((2, 3)), np.zeros((2, 3)))
        S = o.structural_stress()
        assert np.allclose(S, -kT / L ** 3 * weight * np.outer(u, u), rtol=1e-12, atol=1e-30), h


def test_structural_stress_trace_counts_shell_neighbours():
    """Trace = -(kT/V) * 20 * (ordered pairs within the shell), counted here directly."""
    n, L = 300, (16.0, 16.0, 16.0)
    a = gen.radii_bidisperse(n, 3)
    x, v, w = gen.random_state(n, L, a, seed=5)
    kT = 0.8
    o = O.Oracle(_params(L, kT=kT), a, x, v, w)
    S = o.structural_stress()
    d = x[:, None, :] - x[None, :, :]
    d -= np.asarray(L) * np.rint(d / np.asarray(L))
    dist = np.linalg.norm(d, axis=2)
    h = dist - (a[:, None] + a[None, :])
    inshell = (h <= 0.05 * a[:, None]) & ~np.eye(n, dtype=bool)
    assert inshell.sum() > 20
    V = np.prod(L)
    assert math.isclose(np.trace(S), -kT / V * 20.0 * inshell.sum(), rel_tol=1e-12)
    assert np.allclose(S, S.T, rtol=0, atol=1e-15 * np.abs(S).max())


# --------------------------------------------------------------------------
# Rotational lubrication couplings and pairwise Brownian torques (Sec. II.B-II.C)
# --------------------------------------------------------------------------
ROT_ONLY_LUB = O.FREEZE_X | O.NO_PAIR_BROWN | O.NO_CONTACT | O.NO_ONEBODY | O.LUB_ROT


def test_rot_scalars_equal_spheres_and_label_swap():
    eta, xi = 0.1, 0.02
    L = math.log(1 / xi)
    a = 1.3
    YB11, YB21, YC11, YC12, YC21, YC22 = O.lub_rot_scalars(eta, a, a, xi)
    # equal spheres: Y^B = -pi eta a^2 ln(1/xi), Y^C_11 = 1.6 pi eta a^3 ln, Y^C_12 = 0.4 pi eta a^3 ln
    assert math.isclose(YB11, -PI * eta * a * a * L, rel_tol=1e-14) and math.isclose(YB21, YB11, rel_tol=1e-14)
    assert math.isclose(YC11, 1.6 * PI * eta * a ** 3 * L, rel_tol=1e-14) and math.isclose(YC22, YC11, rel_tol=1e-14)
    assert math.isclose(YC12, 0.4 * PI * eta * a ** 3 * L, rel_tol=1e-14) and math.isclose(YC21, YC12, rel_tol=1e-14)
    for ai, aj in ((1.0, 1.4), (0.6, 1.6)):
        y = O.lub_rot_scalars(eta, ai, aj, xi)
        z = O.lub_rot_scalars(eta, aj, ai, xi)
        assert np.allclose([y[1], y[0], y[5], y[4], y[3], y[2]], z, rtol=1e-13, atol=0)
        assert math.isclose(y[3], y[4], rel_tol=1e-13)   # Y^C_12 = Y^C_21


def _pair_state(a, xi, direction, v, w, L=20.0):
    a = np.array(a, float)
    n = np.array(direction, float)
    n /= np.linalg.norm(n)
    sa = a.sum()
    dist = sa * (1 + xi / 2)
    c = np.array([L / 2] * 3)
    return a, np.array([c + 0.5 * dist * n, c - 0.5 * dist * n]), n, dist, c


def test_rigid_rotation_of_a_pair_is_force_free_to_order_h():
    """A pair turning rigidly with the fluid (U_i = Omega x (x_i - c), Omega_i = Omega) is nearly
    free of lubrication force and torque: with the printed scalars F_i = -Y^A h (Omega x n),
    T_i = -Y^B_11 h T Omega, T_j = -Y^B_21 h T Omega, h the gap (n from j to i)."""
    eta = 0.1
    Om = np.array([0.4, -0.7, 0.25])
    for a in ((1.0, 1.0), (1.0, 1.4), (0.6, 1.6)):
        for xi in (2e-3, 0.02):
            a_, x, n, dist, c = _pair_state(a, xi, (0.3, -0.5, 0.8), None, None)
            v = np.cross(Om, x - c)
            w = np.array([Om, Om])
            o = O.Oracle(_params((20.0,) * 3, eta=eta, flags=ROT_ONLY_LUB), a_, x, v, w)
            st = o.state()
            h = dist - a_.sum()
            XA, YA = O.lub_scalars(eta, a_[0], a_[1], xi)
            YB11, YB21 = O.lub_rot_scalars(eta, a_[0], a_[1], xi)[:2]
            TOm = Om - (Om @ n) * n
            scale = YA * dist * np.linalg.norm(Om)
            assert np.abs(st["F"][0] - (-YA * h * np.cross(Om, n))).max() < 1e-12 * scale, (a, xi)
            assert np.abs(st["T"][0] - (-YB11 * h * TOm)).max() < 1e-12 * scale * dist
            assert np.abs(st["T"][1] - (-YB21 * h * TOm)).max() < 1e-12 * scale * dist


def _resistance(a, xi, direction, eta=0.1):
    cols = []
    for k in range(12):
        V = np.zeros(12)
        V[k] = 1.0
        a_, x, n, dist, c = _pair_state(a, xi, direction, None, None)
        o = O.Oracle(_params((20.0,) * 3, eta=eta, flags=ROT_ONLY_LUB), a_, x, V[:6].reshape(2, 3),
                     V[6:].reshape(2, 3))
        st = o.state()
        cols.append(-np.concatenate([st["F"].ravel(), st["T"].ravel()]))
    return np.array(cols).T, n


def test_pair_resistance_symmetric_and_dissipative():
    """The 12x12 matrix taking (U_i, U_j, Omega_i, Omega_j) to -(F_i, F_j, T_i, T_j) is symmetric
    (reciprocal theorem; it fixes the signs of the Y^B couplings in force and torque) and
    positive semi-definite (lubrication only dissipates)."""
    for a in ((1.0, 1.0), (1.0, 1.4), (0.6, 1.6)):
        R, _ = _resistance(a, 0.01, (0.3, -0.5, 0.8))
        assert np.abs(R - R.T).max() <= 1e-13 * np.abs(R).max()
        ev = np.linalg.eigvalsh(0.5 * (R + R.T))
        assert ev.min() >= -1e-12 * ev.max()
        assert np.abs(R[:6, 6:]).max() > 0.01 * np.abs(R).max()   # the couplings are really there


def test_pair_brownian_torques_fluctuation_dissipation():
    """Covariances of the pair's Brownian force and torques over many steps against 2kT/dt times
    the corresponding blocks of the lubrication resistance: <F_i T_i^T> = b^2 R_{F_i Omega_i},
    <T_i T_i^T> = b^2 R_{T_i Omega_i}, <T_j T_j^T> = b^2 R_{T_j Omega_j}."""
    a, xi, kT, dt = (1.0, 1.4), 0.01, 0.5, 1e-4
    R, n = _resistance(a, xi, (0.3, -0.5, 0.8))
    a_, x, n, dist, c = _pair_state(a, xi, (0.3, -0.5, 0.8), None, None)
    o = O.Oracle(_params((20.0,) * 3, kT=kT, dt=dt, seed=21,
                         flags=O.FREEZE_X | O.NO_LUB | O.NO_CONTACT | O.NO_ONEBODY | O.LUB_ROT),
                 a_, x, np.zeros((2, 3)), np.zeros((2, 3)))
    K = 20000
    Fs, Ti, Tj = np.zeros((K, 3)), np.zeros((K, 3)), np.zeros((K, 3))
    for k in range(K):
        o.step(1)
        st = o.state()
        Fs[k], Ti[k], Tj[k] = st["F"][0], st["T"][0], st["T"][1]
    b2 = 2 * kT / dt
    for A, B, target in ((Fs, Ti, R[0:3, 6:9]), (Ti, Ti, R[6:9, 6:9]), (Tj, Tj, R[9:12, 9:12])):
        est = A.T @ B / K
        # standard error of each entry of a mean of products: sqrt((<a^2><b^2> + <ab>^2) / K)
        va, vb = (A * A).mean(axis=0), (B * B).mean(axis=0)
        se = np.sqrt((np.outer(va, vb) + est * est) / K)
        assert (np.abs(est - b2 * target) < 6 * se + 1e-12 * b2 * np.abs(target).max()).all(), (est / b2, target)
    assert (np.abs(Ti.mean(axis=0)) < 6 * np.sqrt((Ti * Ti).mean(axis=0) / K)).all()


# --------------------------------------------------------------------------
# Trajectory analysis: non-affine displacement, pair-distance histogram
# --------------------------------------------------------------------------
def test_displacement_of_a_free_particle_in_shear():
    """A force-free particle starting with the local flow velocity and moving across y drifts
    away from the flow by exactly -gammadot v_y t^2 / 2 along x (wrapping through the sheared
    boundary changes nothing), and by v_y t along y."""
    L, gd, vy, dt = 12.0, 0.8, 3.0, 1e-3
    y0 = 10.5
    x = np.array([[5.0, y0, 6.0], [1.0, 1.0, 1.0]])
    a = np.array([1.0, 1.0])
    v = np.array([[gd * (y0 - L / 2), vy, 0.0], [gd * (1.0 - L / 2), 0.0, 0.0]])
    o = O.Oracle(_params((L, L, L), gammadot=gd, dt=dt, flags=O.NO_ONEBODY | O.NO_PAIR_BROWN), a, x, v, np.zeros((2, 3)))
    nsteps = 1000                     # crosses y = L after ~500 steps
    o.step(nsteps)
    t = nsteps * dt
    d = o.displacement()
    assert o.state()["x"][0, 1] < y0   # it went through the boundary
    assert math.isclose(d[0, 0], -0.5 * gd * vy * t * t, rel_tol=1e-10)
    assert math.isclose(d[0, 1], vy * t, rel_tol=1e-12) and d[0, 2] == 0.0
    assert np.abs(d[1]).max() < 1e-15   # the second sphere rides with the flow


def test_displacement_matches_positions_modulo_box():
    """Without shear the accumulated displacement is the unwrapped motion: positions change by
    it modulo the box."""
    n, L = 200, (14.0, 14.0, 14.0)
    a = gen.radii_bidisperse(n, 8)
    x, v, w = gen.random_state(n, L, a, seed=9, kT=4.0)
    o = O.Oracle(_params(L, kT=4.0, dt=2e-4, seed=3, flags=O.NO_CONTACT), a, x, v, w)
    o.step(300)
    d = o.displacement()
    jump = (o.state()["x"] - x - d) / np.asarray(L)
    assert np.abs(jump - np.rint(jump)).max() < 1e-10
    assert np.abs(d).max() > 1e-3


def test_rdf_histogram_brute_force():
    n, L = 300, (13.0, 13.0, 13.0)
    a = gen.radii_bidisperse(n, 5)
    x, v, w = gen.random_state(n, L, a, seed=6)
    o = O.Oracle(_params(L), a, x, v, w)
    r_max, nb = 3.0, 30
    h = o.rdf(r_max, nb)
    d = x[:, None, :] - x[None, :, :]
    d -= np.asarray(L) * np.rint(d / np.asarray(L))
    r = np.linalg.norm(d, axis=2)[np.triu_indices(n, 1)]
    ref, _ = np.histogram(r[r < r_max], bins=nb, range=(0.0, r_max))
    assert h.sum() == ref.sum() > 100
    assert np.abs(h.astype(np.int64) - ref).sum() <= 2   # a distance on a bin edge may round either way


# --------------------------------------------------------------------------
# Drag stresslet, total stress and relative viscosity (Sec. II.B, II.E, IV.D)
# --------------------------------------------------------------------------
def test_drag_stresslet_is_einstein_viscosity():
    """Sec. II.B gives each particle the drag stress (20/3) pi eta a^3 E with E_xy = gammadot/2;
    summed over a volume V this is 2.5 phi eta gammadot, Einstein's dilute-suspension result
    (phi = sum (4/3) pi a^3 / V).  A dilute system without pairs in range has no pair stress, so
    its total stress (Sec. IV.D) is the drag stresslet and eta_r = 2.5 phi exactly."""
    for n, L, gd in ((40, (60.0, 55.0, 70.0), 0.3), (500, (19.9, 19.9, 19.9), 0.53)):
        a = gen.radii_bidisperse(n, 1)
        V = float(np.prod(L))
        phi = float(np.sum(4.0 / 3.0 * PI * a ** 3) / V)
        if n == 40:   # spheres on a coarse lattice: no pair within the cut-off
            g = np.stack(np.meshgrid(np.arange(4), np.arange(2), np.arange(5), indexing="ij"), -1).reshape(-1, 3)
            x = (g + 0.5) * np.array([L[0] / 4, L[1] / 2, L[2] / 5])
        else:
            x = gen.relaxed_positions(a, L[0], 3)
        v = np.zeros((n, 3))
        w = np.zeros((n, 3))
        o = O.Oracle(_params(L, gammadot=gd, kT=0.0, eta=0.1), a, x, v, w)
        S = o.stress_all()
        eta = 0.1
        assert S[3][0, 1] / (eta * gd) == pytest.approx(2.5 * phi, rel=1e-12)
        assert S[3][1, 0] == S[3][0, 1]
        mask = np.ones((3, 3), bool)
        mask[0, 1] = mask[1, 0] = False
        assert np.all(S[3][mask] == 0.0)
        # total = hydrodynamic (lubrication + drag) + contact; Brownian excluded
        assert np.allclose(S[4], S[0] + S[1] + S[3], rtol=1e-15, atol=0)
        assert o.eta_r() == pytest.approx(S[4][0, 1] / (eta * gd), rel=1e-15)
        if n == 40:
            assert len(o.pairs()) == 0 and np.all(S[:3] == 0.0)
            assert o.eta_r() == pytest.approx(2.5 * phi, rel=1e-12)
    # no one-body terms, no drag stresslet
    o = O.Oracle(_params(L, gammadot=0.3, flags=O.NO_ONEBODY), a, x, v, w)
    assert np.all(o.stress_all()[3] == 0.0)


def test_single_sphere_relaxes_to_imposed_flow():
    """One sphere, kT = 0, at rest in shear flow.  With the drag of eq. (force_drag) and
    (torque_drag) evaluated at the half-step velocities of velocity-Verlet, the departure
    u = v - U^inf(x) of the full-step velocity obeys u_n = (1 - c)^2 (1 - 2c)^(n-1) u_0 with
    c = zeta dt / (2 m), zeta = 6 pi eta a, m = (4/3) pi rho a^3 (Sec. II), and likewise the
    spin relaxes towards Omega^inf = (1/2) curl U^inf with c_r = zeta_r dt / (2 I), zeta_r =
    8 pi eta a^3, I = (2/5) m a^2.  The limits pin the gauge U^inf = gammadot (y - Ly/2) e_x and
    the sign of Omega^inf; the rates pin zeta, zeta_r, m and I; the discrete law pins the
    kick-drift-kick order.  (Continuous-time limit: exp(-zeta t / m).)"""
    L = (12.0, 10.0, 11.0)
    gd, eta, rho, dt, a = 0.7, 0.1, 0.1, 1e-4, 1.3
    y0 = 0.8 * L[1]
    x = np.array([[3.0, y0, 5.0]])
    v0 = np.array([[0.05, 0.0, -0.02]])
    w0 = np.array([[0.1, -0.3, 0.2]])
    o = O.Oracle(_params(L, gammadot=gd, kT=0.0, eta=eta, rho=rho, dt=dt), np.array([a]), x, v0, w0)
    # imposed flow at the sphere and its vorticity, from U^inf(x) = gammadot (y - Ly/2) e_x
    U = np.array([gd * (y0 - 0.5 * L[1]), 0.0, 0.0])
    dUx_dy, dUy_dx = gd, 0.0
    Om = np.array([0.0, 0.0, 0.5 * (dUy_dx - dUx_dy)])
    m = 4.0 / 3.0 * PI * rho * a ** 3
    I = 0.4 * m * a ** 2
    c = 6 * PI * eta * a * dt / (2 * m)
    cr = 8 * PI * eta * a ** 3 * dt / (2 * I)
    done = 0
    for nsteps in (1, 10, 300, 2000):
        o.step(nsteps - done)
        done = nsteps
        st = o.state()
        fac = (1 - c) ** 2 * (1 - 2 * c) ** (nsteps - 1)
        facr = (1 - cr) ** 2 * (1 - 2 * cr) ** (nsteps - 1)
        assert np.allclose(st["v"][0] - U, fac * (v0[0] - U), rtol=1e-11, atol=1e-17)
        assert np.allclose(st["w"][0] - Om, facr * (w0[0] - Om), rtol=1e-11, atol=1e-17)
        assert st["x"][0, 1] == y0    # no gradient-direction motion
    assert abs(st["w"][0, 2] - Om[2]) < 0.25 * abs(w0[0, 2] - Om[2])   # relaxed towards -gammadot / 2


# --------------------------------------------------------------------------
# Two-sphere potential of mean force (Sec. III.A)
# --------------------------------------------------------------------------
_PMF_EDGES = np.linspace(0.0, 2.5, 251)


def _pmf_counts(flags, seeds, kn, nsteps=2_000_000):
    """Two spheres of radius 1 in a periodic box of side 5 without flow; pair-distance
    histogram every 5 steps over independent runs (threads: the oracle releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    x = np.array([[1.0, 1.0, 1.0], [3.5, 3.5, 3.5]])
    z = np.zeros((2, 3))
    O.lib()

    def one(seed):
        o = O.Oracle(_params((5.0, 5.0, 5.0), kn=kn, kt=2 * kn / 7, kT=1.0, gammadot=0.0, seed=seed, flags=flags),
                     np.ones(2), x, z, z)
        return o.run_rdf(nsteps, 5, 2.5, len(_PMF_EDGES) - 1)

    with ThreadPoolExecutor(8) as ex:
        return sum(ex.map(one, seeds))


def _pmf_ratios(counts, kn, regions):
    """Observed counts over those of g(r) = exp(-U(r)/kT), U = (1/2) k_n delta^2 in contact and
    0 outside (the potential of mean force the paper reports), per region of r; the
    histogram is normalised on 2.05 <= r <= 2.45 (r < L/2: whole spherical shells)."""
    def shell(lo, hi):
        r = np.linspace(lo, hi, 201)
        return np.trapezoid(4 * PI * r ** 2 * np.exp(-0.5 * kn * np.clip(2.0 - r, 0, None) ** 2), r)

    lo_e, hi_e = _PMF_EDGES[:-1], _PMF_EDGES[1:]

    def region(lo, hi):
        k = np.where((lo_e >= lo - 1e-12) & (hi_e <= hi + 1e-12))[0]
        return counts[k].sum(), sum(shell(lo_e[q], hi_e[q]) for q in k)

    c0, e0 = region(2.05, 2.45)
    out = []
    for lo, hi in regions:
        c, e = region(lo, hi)
        out.append(float(c / (e * c0 / e0)))
    return out


@pytest.mark.slow
def test_two_sphere_pmf_contact_potential():
    """Contact force and one-body thermostat alone (Sec. III.A): inside contact -ln g(r) =
    (1/2) k_n delta^2 / kT, outside it g is flat (k_n = 300, kT = 1: delta_rms ~ 0.06)."""
    kn = 300.0
    rat = _pmf_ratios(_pmf_counts(O.NO_LUB | O.NO_PAIR_BROWN, range(16), kn), kn,
                      [(1.8, 1.9), (1.9, 2.0), (2.0, 2.05), (2.05, 2.25), (2.25, 2.45)])
    assert abs(rat[0] - 1) < 0.3 and abs(rat[1] - 1) < 0.15, rat
    assert all(abs(t - 1) < 0.08 for t in rat[2:]), rat


@pytest.mark.slow
def test_two_sphere_pmf_flat_outside_contact():
    """All forces (Sec. III.A): lubrication and the pairwise Brownian force introduce no net
    potential outside contact, so g(r) is flat for r > 2a, also inside the lubrication range
    2a < r < 2.05a where they act.  (Inside contact, with dt = 1e-4, the lubricated pair
    samples its overlap in long, rare episodes: that region is not asserted.)"""
    kn = 300.0
    rat = _pmf_ratios(_pmf_counts(0, range(100, 116), kn), kn, [(2.0, 2.05), (2.05, 2.25), (2.25, 2.45)])
    assert all(abs(t - 1) < 0.04 for t in rat), rat


# --------------------------------------------------------------------------
# Stress autocorrelation (the Green-Kubo integrand of Sec. IV.B)
# --------------------------------------------------------------------------
def test_acf_closed_forms():
    """Series with closed-form autocorrelations: a constant c gives c^2 at every lag; the
    alternating series (-1)^t gives (-1)^k exactly; a series and its time reverse give the
    same estimator; lag 0 is the mean square; AR(1) noise decays as phi^k."""
    assert np.array_equal(O.acf(np.full(50, 3.0), 10), np.full(10, 9.0))
    alt = np.array([(-1.0) ** t for t in range(101)])
    assert np.array_equal(O.acf(alt, 20), np.array([(-1.0) ** k for k in range(20)]))
    rng = np.random.default_rng(5)
    s = rng.normal(size=300)
    c = O.acf(s, 40)
    assert np.allclose(c, O.acf(s[::-1], 40), rtol=1e-13, atol=1e-15)
    assert c[0] == pytest.approx(np.mean(s * s), rel=1e-14)
    assert np.array_equal(O.acf(s, 400)[300:], np.zeros(100))
    # AR(1): s_t = phi s_(t-1) + e_t, stationary variance 1 / (1 - phi^2)
    ph, n = 0.8, 400_000
    e = rng.normal(size=n)
    ar = np.empty(n)
    ar[0] = e[0] / math.sqrt(1 - ph * ph)
    for t in range(1, n):
        ar[t] = ph * ar[t - 1] + e[t]
    c = O.acf(ar, 8)
    assert np.allclose(c, ph ** np.arange(8) / (1 - ph * ph), rtol=0.05)


def test_rdf_xy_slice_brute_force():
    """The flow-gradient slice of the pair distribution against a numpy enumeration of all pairs
    in an unsheared box: identical counts (up to bin-edge rounding), point-symmetric."""
    n, L = 250, (12.0, 12.5, 13.0)
    a = gen.radii_bidisperse(n, 5)
    x, v, w = gen.random_state(n, L, a, seed=7)
    o = O.Oracle(_params(L), a, x, v, w)
    r_max, slab, nb = 4.0, 1.5, 16
    h = o.rdf_xy(r_max, slab, nb)
    d = x[:, None, :] - x[None, :, :]
    d -= np.asarray(L) * np.rint(d / np.asarray(L))
    iu = np.triu_indices(n, 1)
    r = d[iu]
    sel = (np.abs(r[:, 2]) < slab / 2) & (np.abs(r[:, 0]) < r_max) & (np.abs(r[:, 1]) < r_max)
    r = r[sel]
    both = np.concatenate([r[:, :2], -r[:, :2]])
    ref, _, _ = np.histogram2d(both[:, 0], both[:, 1], bins=nb, range=((-r_max, r_max), (-r_max, r_max)))
    assert h.sum() == ref.sum() > 200
    assert np.abs(h.astype(np.int64) - ref.astype(np.int64)).sum() <= 4
    assert np.array_equal(h, h[::-1, ::-1])
