"""tnn_query_noalloc (the entry point that takes no scratch buffer) against
tnn_query on the same inputs: two calls in a row, the second with fewer
queries and a smaller index, every flag combination that fits the library's
per-device scratch; and the size limit.  Through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, build, dev_points, say
from paper_2112_10408_amd import capi, synth
from paper_2112_10408_amd import tnn as T

pytestmark = pytest.mark.gpu

FLAGS = [("plain", capi.TNN_PLAIN), ("learned", capi.TNN_LEARNED), ("brute", capi.TNN_BRUTE),
         ("bf16", capi.TNN_BRUTE | capi.TNN_MIXED_BF16)]


def _run_both(ix, qs, k, tw, flags, model):
    q = dev_points(qs)
    r2 = T.tnn_radius_infer(model, *q, alpha=1.5) if flags & capi.TNN_LEARNED else None
    gi, gd = T.tnn_query(ix, *q, synth.SCALE, tw, k, flags=flags, radius2=r2)
    ni, nd = T.tnn_query_noalloc(ix, *q, synth.SCALE, tw, k, flags=flags, radius2=r2)
    torch.cuda.synchronize()
    return (gi.cpu().numpy(), gd.cpu().numpy()), (ni.cpu().numpy(), nd.cpu().numpy())


@pytest.mark.parametrize("name,flags", FLAGS, ids=[f[0] for f in FLAGS])
def test_noalloc_matches_tnn_query_twice(name, flags):
    big = synth.trajectories(300, 60, 600.0, 3 * 3600.0, seed=31)
    small = synth.trajectories(40, 30, 200.0, 3600.0, seed=32)
    cases = [(big, 3000, 16, 32, 0.0), (small, 400, 8, 8, 60.0)]
    for step, (ps, nq, K, k, tw) in enumerate(cases):
        say(f"no-alloc {name} call {step}: {ps.n} points, {nq} queries, K={K}, k={k}, t_w={tw}")
        ix = build(ps, K)
        model = T.tnn_radius_model_init(ix, seed=3)
        qs, _ = synth.sample_queries(ps, nq, seed=40 + step)
        (gi, gd), (ni, nd) = _run_both(ix, qs, k, tw, flags, model)
        # the existing entry point and the new one agree bit for bit
        assert np.array_equal(gi, ni) and np.array_equal(gd, nd), f"{name} call {step}"
        # and both meet the oracle (indices exact, distances the oracle's)
        oi, od = oracle.knn(ps.soa(), qs.soa(), synth.SCALE, tw, k)
        assert_same(ni, nd, oi, od, f"no-alloc {name} call {step}")


def test_noalloc_rejects_scratch_beyond_its_limit():
    """The BF16 linear search needs 64 B per point: a 300k-point index is
    beyond the library's 16 MiB, which is reported before anything runs (the
    outputs keep their contents); the TNN path of the same index fits."""
    ps = synth.trajectories(1500, 200, 3000.0, 12 * 3600.0, seed=33)
    ix = build(ps, 32)
    qs, _ = synth.sample_queries(ps, 256, seed=34)
    q = dev_points(qs)
    mf = capi.TNN_BRUTE | capi.TNN_MIXED_BF16
    need = T.tnn_query_workspace(ix, qs.n, T.make_params(synth.SCALE, 0.0, 8, mf))
    assert need > capi.NOALLOC_SCRATCH_BYTES
    out = (torch.full((qs.n, 8), 7, dtype=torch.int32, device="cuda"),
           torch.full((qs.n, 8), 3.0, dtype=torch.float64, device="cuda"))
    with pytest.raises(capi.TnnError) as e:
        T.tnn_query_noalloc(ix, *q, synth.SCALE, 0.0, 8, flags=mf, out=out)
    assert e.value.code == capi.TNN_E_WORKSPACE
    torch.cuda.synchronize()
    assert bool((out[0] == 7).all()) and bool((out[1] == 3.0).all())
    ni, nd = T.tnn_query_noalloc(ix, *q, synth.SCALE, 0.0, 8)
    gi, gd = T.tnn_query(ix, *q, synth.SCALE, 0.0, 8)
    torch.cuda.synchronize()
    assert torch.equal(ni, gi) and torch.equal(nd, gd)
