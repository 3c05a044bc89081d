"""The entry point that allocates no device memory (fixed workspace):
through the C ABI it gives exactly bp_partition_device's results, on two calls
in a row with the second input smaller, leaves the device's free memory
unchanged, and refuses an input too large for the workspace with
BP_ERR_OUT_OF_MEMORY before doing any work."""
import sys

import numpy as np
import pytest

import oracle
from paper_2012_13618_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_13618_amd as mod
    mod.lib()
    return mod


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(bp, h, k, eps, prm=None):
    import torch
    dh = bp.DeviceHypergraph.from_host(h)
    a = torch.full((h.num_nodes,), -1, dtype=torch.int32, device="cuda")
    b = torch.full((h.num_nodes,), -2, dtype=torch.int32, device="cuda")
    _, cut_a, st_a, rep_a = bp.partition_device(dh, k, eps, prm=prm, part_out=a)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    _, cut_b, st_b, rep_b = bp.partition_device_noalloc(dh, k, eps, prm=prm, part_out=b)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return a.cpu().numpy(), cut_a, st_a, b.cpu().numpy(), cut_b, st_b, rep_b, free0, free1


def test_noalloc_equals_partition_device_twice(bp):
    cases = [(I.vlsi(seed=31, n=20000), 4, 0.05), (I.tiny(), 2, 0.05)]
    for i, (h, k, eps) in enumerate(cases):
        say(f"call {i}: N={h.num_nodes} P={h.num_pins} k={k}")
        a, ca, sa, b, cb, sb, rep, f0, f1 = _both(bp, h, k, eps)
        assert np.array_equal(a, b) and ca == cb and sa == sb, i
        ref_part, ref_cut = oracle.partition_hg(h, k=k, eps=eps)
        assert np.array_equal(b, ref_part) and cb == ref_cut, i
        say(f"  workspace used {rep.device_bytes} bytes; device free {f0} -> {f1}")
        assert 0 < rep.device_bytes <= 256 << 20
        if i > 0:
            assert f1 == f0


def test_noalloc_params_and_k1(bp):
    h = I.random_small(3000, 3600, 2, 9, 3, weighted_nodes=True, weighted_hedges=True)
    prm = bp.params(policy=bp.HDH, min_coarse_nodes=0)
    a, ca, _, b, cb, _, _, _, _ = _both(bp, h, 5, 0.1, prm=prm)
    assert np.array_equal(a, b) and ca == cb
    a, ca, _, b, cb, _, _, _, _ = _both(bp, h, 1, 0.1)
    assert np.all(b == 0) and cb == 0


def test_noalloc_refuses_oversized_input(bp):
    import torch
    h = I.vlsi()
    dh = bp.DeviceHypergraph.from_host(h)
    out = torch.empty(h.num_nodes, dtype=torch.int32, device="cuda")
    with pytest.raises(bp.BipartError) as ei:
        bp.partition_device_noalloc(dh, 2, 0.05, part_out=out)
    assert ei.value.status == -4 and "workspace" in str(ei.value)
    # still usable afterwards
    small = I.tiny()
    a, ca, _, b, cb, _, _, _, _ = _both(bp, small, 2, 0.05)
    assert np.array_equal(a, b) and ca == cb
