"""The near-degenerate input recipe (tests/near_degenerate.py) produces, in
every family, pairs on both sides of the decision (shared vertices always
touch), so the GPU falsification test exercises both answers of each
boundary case.  CPU only."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import near_degenerate as nd  # noqa: E402


def test_every_family_has_both_outcomes(oracle_mod):
    T, U, F = nd.make_pairs(3000, seed=5)
    A, B = nd.as_meshsets(T, U)
    pairs = np.stack([np.arange(T.shape[0])] * 2, 1).astype(np.int32)
    f = oracle_mod.join(A, B, pairs, mode=0)
    for k, name in enumerate(nd.FAMILIES):
        m = F == k
        assert m.sum() > 200, name
        assert f[m].sum() > 0, name
        if name != "shared_vertex":
            assert f[m].sum() < m.sum(), name
    # some pairs lie outside the FP32-bound range, most inside
    mag = np.abs(np.concatenate([T.reshape(-1), U.reshape(-1)]))
    mag = mag[mag > 0]
    assert (mag < 2.0 ** -40).any() or (mag > 2.0 ** 40).any()
    assert np.mean((mag >= 2.0 ** -40) & (mag <= 2.0 ** 40)) > 0.9
