"""The entry point that allocates nothing: sim_rdf_noalloc, called through the C ABI, against
sim_rdf on the same state, on two calls in a row (the second with fewer bins and a shorter
range, so that stale counts of the first would show), and rejected beyond its array."""
import ctypes as C
import sys

import numpy as np
import pytest

from inputs import gen

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_rdf_noalloc_matches_rdf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_13802_amd as P
    from paper_2307_13802_amd import sim as S
    L = P.lib()
    st = gen.make_state(gen.Workload("t", 3000, 0.55, 10.0, seed=41))
    # count the library's allocations through the allocator hook
    calls = []

    def _alloc(nbytes, ctx):
        calls.append(int(nbytes))
        return int(torch.cuda.caching_allocator_alloc(int(nbytes)))

    def _free(p, ctx):
        torch.cuda.caching_allocator_delete(p)

    a, f = S._ALLOC_CB(_alloc), S._FREE_CB(_free)
    assert L.sim_set_allocator(a, f, None) == 0
    try:
        sim = P.Sim(P.Config(box=st["L"], **st["params"]), st["radii"], st["x"], st["v"], st["w"])
        sim.step(50)
        for r_max, nb in ((7.5, 3000), (4.0, 37)):
            _say(f"case: sim_rdf_noalloc r_max={r_max} bins={nb}, N=3000")
            before = len(calls)
            got = np.zeros(nb, np.uint64)
            rc = L.sim_rdf_noalloc(sim.h, 0, r_max, nb, got.ctypes.data_as(C.POINTER(C.c_uint64)))
            assert rc == 0, P.sim._err(sim.h)
            assert len(calls) == before   # nothing allocated through the library
            ref = sim.rdf(r_max, nb)      # the allocating entry point on the same state
            assert got.sum() > 1000 and np.array_equal(got, ref)
        bad = np.zeros(70000, np.uint64)
        assert L.sim_rdf_noalloc(sim.h, 0, 4.0, 70000, bad.ctypes.data_as(C.POINTER(C.c_uint64))) == P.sim.EINVAL
        assert "65536" in P.sim._err(sim.h)
        sim.close()
    finally:
        P.use_default_allocator()
