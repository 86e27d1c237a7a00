"""tn_distance_noalloc (the allocation-free distance entry point, whose
workspace is the library's fixed device array) against tn_distance with a
caller workspace: the same kernels, so the same bits, on two calls in a row
(the second on a smaller population, reusing the array the first one filled),
and a population beyond the array's size is refused before anything runs."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import host, to_device

pytestmark = pytest.mark.gpu


def _bits(t):
    return host(t).view(np.uint32)


def _both(pop):
    import paper_2504_08339_amd as tn
    dp = to_device(pop)
    ref = tn.distance(dp, 1.0, 1.0, 0.4)
    got = tn.distance_noalloc(dp, 1.0, 1.0, 0.4)
    return ref, got


def test_noalloc_equals_workspace_form_twice_smaller_second():
    first = synth.control_population(P=700)
    second = synth.subset(synth.batching_population(P=200), list(range(0, 200, 2)))
    for pop in (first, second):
        (d0, e0, f0), (d1, e1, f1) = _both(pop)
        assert np.array_equal(_bits(d1), _bits(d0))
        assert np.array_equal(host(e1), host(e0))
        assert np.array_equal(host(f1), host(f0))
    # the second result is the second population's, not left over from the first
    assert host(d1).shape == (second.P, second.P)


def test_noalloc_without_counts_and_into_given_outputs():
    import paper_2504_08339_amd as tn
    pop = synth.control_population(P=150)
    dp = to_device(pop)
    ref, _, _ = tn.distance(dp, 1.0, 1.0, 0.4, counts=False)
    out = (torch.empty((pop.P, pop.P), dtype=torch.float32, device="cuda"),
           torch.empty((pop.P, pop.P), dtype=torch.int32, device="cuda"),
           torch.empty((pop.P, pop.P), dtype=torch.int32, device="cuda"))
    d, e, f = tn.distance_noalloc(dp, 1.0, 1.0, 0.4, out=out)
    assert d.data_ptr() == out[0].data_ptr()
    assert np.array_equal(_bits(d), _bits(ref))
    d2, e2, f2 = tn.distance_noalloc(dp, 1.0, 1.0, 0.4, counts=False)
    assert e2 is None and f2 is None
    assert np.array_equal(_bits(d2), _bits(ref))


def test_noalloc_refuses_population_beyond_scratch():
    import paper_2504_08339_amd as tn
    P, N, C = 4096, 8, 1024                    # workspace 4096 * 1024 * 16 B = 64 MiB
    arrays = {
        "node_key": np.full((P, N), -1, np.int32), "node_bias": np.zeros((P, N), np.float32),
        "node_resp": np.ones((P, N), np.float32), "node_act": np.zeros((P, N), np.uint8),
        "node_agg": np.zeros((P, N), np.uint8), "conn_in": np.full((P, C), -1, np.int32),
        "conn_out": np.full((P, C), -1, np.int32), "conn_w": np.zeros((P, C), np.float32),
        "conn_en": np.zeros((P, C), np.uint8),
    }
    dp = tn.Population.from_numpy(2, 1, N, C, arrays, device="cuda")
    with pytest.raises(tn.TNError) as e:
        tn.distance_noalloc(dp)
    assert e.value.code == 3                   # TN_EUNSUPPORTED
    # the workspace form still takes it
    d, E, D = tn.distance(dp, counts=True)
    assert np.all(host(E)[:4, :4] == 0)
