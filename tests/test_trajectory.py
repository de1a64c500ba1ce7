"""Trajectory parity: the HIP path against the FP64 oracle over whole runs.

Both sides integrate the same initial state with the same Philox keys, so they
follow the same trajectory until rounding differences, amplified by the
dynamics, change the interaction set.  At each checkpoint: the interaction set
(bit-exact), the positions, and the per-step stress series of the chunk; at the
end, the mean pair shear stress (contact + lubrication + Brownian, xy) against
the oracle's, beside its block standard error.

The 1,000-step run of the 500-sphere workload and the 2,000-step prefix of the
50,000-sphere workload (about two minutes of oracle time) both run with the GPU
tests.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from inputs import gen

pytestmark = pytest.mark.gpu

# margins of 100x and more over what the MI355X shows (positions 3e-13, stress 3e-11)
TOL_X = 1e-10
TOL_STRESS = 1e-8
TOL_MEAN = 1e-10


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


def _pair_xy(series):
    """Per-step shear stress xy summed over the three kinds, from (steps, 27) records."""
    return series.reshape(-1, 3, 3, 3)[:, :, 0, 1].sum(axis=1)


def _run(P, w, chunks, chunk, cells):
    st = gen.make_state(w)
    n = len(st["radii"])
    sim = P.Sim(P.Config(box=st["L"], precision=P.FP64, **st["params"]), st["radii"], st["x"], st["v"], st["w"])
    orc = O.Oracle(O.Params(L=st["L"], **st["params"], flags=(O.CELLS if cells else 0)), st["radii"], st["x"],
                   st["v"], st["w"])
    sg_all, so_all = [], []
    for c in range(chunks):
        sim.step(chunk)
        sg = sim.stress_series().reshape(-1, 27)
        so = orc.step(chunk, series=True)
        g, o = sim.get_state(), orc.state()
        same = np.array_equal(sim.pairs(), orc.pairs())
        dx = float(np.abs(g["x"] - o["x"]).max())
        ds = float((np.abs(sg - so) / (np.abs(so).max(axis=0) + 1e-300)).max())
        _say(f"  N={n} step {(c + 1) * chunk}: same interaction set {same}, max |dx| {dx:.2e}, "
             f"stress series max rel diff {ds:.2e}")
        assert same, f"interaction sets differ at step {(c + 1) * chunk}"
        assert g["step"] == o["step"] and g["s_le"] == o["s_le"]
        assert sg.shape == so.shape
        assert dx < TOL_X and ds < TOL_STRESS
        sg_all.append(sg)
        so_all.append(so)
    xg, xo = _pair_xy(np.concatenate(sg_all)), _pair_xy(np.concatenate(so_all))
    mg, mo = float(xg.mean()), float(xo.mean())
    blocks = xo[: len(xo) // 10 * 10].reshape(10, -1).mean(axis=1)
    se = float(blocks.std(ddof=1) / np.sqrt(10))
    rel = (mg - mo) / abs(mo)
    _say(f"  N={n}, {chunks * chunk} steps: mean pair shear stress GPU {mg:.9e}, oracle {mo:.9e}, "
         f"rel diff {rel:.2e} (block standard error {se / abs(mo):.2e})")
    assert abs(rel) < TOL_MEAN


def test_c1_trajectory_1000_steps(P):
    """500 bidisperse spheres, phi = 0.50, Pe = 1: the whole 1,000-step run."""
    _say("case: trajectory N=500 phi=0.5 Pe=1, 1000 steps in chunks of 100")
    _run(P, gen.C1, 10, 100, cells=False)


def test_c2_prefix_2000_steps(P):
    """50,000 bidisperse spheres, phi = 0.55, Pe = 10: the first 2,000 steps."""
    _say("case: trajectory N=50000 phi=0.55 Pe=10, 2000 steps in chunks of 200")
    _run(P, gen.C2, 10, 200, cells=True)
