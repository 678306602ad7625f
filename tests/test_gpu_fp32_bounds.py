"""Falsification of the FP32 error bounds through refine_intersects.

10^5 pairs of one-triangle meshes built at decision boundaries (vertices
rounded onto planes and edge lines, shared vertices, crossing edges,
axis-parallel edges, exact and near coplanarity, far translations, scales
2^-40..2^40 and a few beyond; tests/near_degenerate.py).  A bound that is
too tight would certify a wrong sign and flip a flag; the slab slack being
too small would prune a touching box.  Both precision modes must give the
oracle's flags bit for bit, and every decision tier must be used: certain
FP32 decisions, FP32-uncertain tests certified by the FP64 filter, and
tests that need exact expansions."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import near_degenerate as nd  # noqa: E402

pytestmark = pytest.mark.gpu


def test_fp32_bounds_never_flip_a_flag():
    import torch
    import oracle
    import paper_2609_24513_amd as pa
    T, U, F = nd.make_pairs(100_000, seed=77)
    A, B = nd.as_meshsets(T, U)
    pairs = np.stack([np.arange(T.shape[0])] * 2, 1).astype(np.int32)
    want = oracle.join(A, B, pairs, mode=0)
    assert 0.2 < want.mean() < 0.8
    for w, leaf in ((4, 4), (2, 1)):
        ga = pa.MeshBlob.build(A, width=w, leaf_size=leaf)
        gb = pa.MeshBlob.build(B, width=w, leaf_size=leaf)
        for prec in (0, 1):
            flags, stats, status = pa.refine(ga, gb, pairs, pa.RefineConfig(precision=prec))
            torch.cuda.synchronize()
            assert int(status.item()) == 0
            got = flags.cpu().numpy()
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, [(int(i), nd.FAMILIES[F[i]], int(want[i])) for i in bad[:10]]
            st = pa.stats_dict(stats)
            if prec == 0:
                assert st["tri_tests"] > st["fp32_ambiguous"] > 1000, st     # certain FP32 decisions
                assert st["exact_decided"] > st["fp64_filter_ambiguous"], st  # FP64 filter certifies some
                assert st["fp64_filter_ambiguous"] > 100, st                 # exact expansions needed
            else:
                assert st["exact_decided"] == st["tri_tests"] > 0, st
        for k, name in enumerate(nd.FAMILIES):   # every family carries both answers
            m = F == k
            assert want[m].sum() > 0, name
