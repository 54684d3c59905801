"""The entry point that allocates nothing (sdem_init_static): a context on the
library's static device scratch steps exactly like one on a caller
workspace (same kernels, same data), twice in a row on one GPU, the second
time with a smaller system on the scratch the first one left behind."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def run(w, static, steps=80):
    from paper_2507_12610_amd import Solver
    s = Solver(w, device="cuda:0", static_scratch=static, skin=0.1)
    s.step(steps)
    out = (s.state(), s.contacts(), s.stats())
    s.close()
    return out


def box_cluster(n, seed, box):
    w = W.random_cluster(n, seed, box=box, overlap=0.15,
                         tri=W.cube_mesh([-0.2e-3] * 3, [box + 0.2e-3] * 3))
    w["params"]["g"] = (0.0, 0.0, -9.81)
    return w


def test_static_scratch_matches_caller_workspace():
    for n, seed, box in ((900, 21, 24e-3), (250, 22, 15e-3)):  # then a smaller system
        w = box_cluster(n, seed, box)
        sa, ca, ta = run(w, static=False)
        sb, cb, tb = run(w, static=True)
        assert len(ca["ki"]) > n // 4, "the case must have contacts"
        assert np.array_equal(ca["ki"], cb["ki"]) and np.array_equal(ca["kj"], cb["kj"]), n
        for k in ("us", "ur", "ut"):
            assert np.array_equal(ca[k], cb[k]), (n, k)
        for k in ("x", "v", "w", "q", "F", "T"):
            assert np.array_equal(sa[k], sb[k]), (n, k)
        assert ta == tb, n


def test_static_scratch_rejects_large_capacities():
    from paper_2507_12610_amd import Solver
    from paper_2507_12610_amd.sdem import SdemError
    w = W.cfg4_sim(0, 60000)
    with pytest.raises(SdemError) as e:
        Solver(w, device="cuda:0", static_scratch=True)
    assert "static scratch" in str(e.value)
