"""The oracle built with OpenMP (used for the CPU baseline's many-core leg
and for long oracle runs in the GPU parity tests) computes every value bit
for bit as the single-threaded build: only loops whose iterations touch
disjoint sites run in parallel, and sums over sites stay serial."""
import numpy as np
import pytest

import gpu_cases as G
import oracle


@pytest.mark.parametrize("name", ["slab_4x4x34", "coax_16x16x4", "random_6x10x14_k3",
                                  "random_8x6x10_k4"])
def test_threaded_oracle_is_bitwise_the_serial_one(name):
    kw, shape, t, ps, n0, nref, nsteps, _ = G.case(name)
    runs = []
    for threads in (None, 4):
        o = oracle.Oracle(oracle.make_params(shape, **kw, tol=1e-12, max_iter=10**6,
                                             check_every=4), t, ps, n0, nref, threads=threads)
        o.step(nsteps)
        runs.append((o.fields(), o.qhist(), o.last_iters, o.threads))
    (fa, qa, ia, ta), (fb, qb, ib, tb) = runs
    assert ta == 1 and tb == 4
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert np.array_equal(qa, qb) and ia == ib
