"""The entry point that allocates nothing (det_mod_primes_noalloc): through
the C ABI, its residues equal det_mod_primes' on the FP64 path, bit for bit,
on consecutive calls that reuse the library's static device array (the second
with a smaller input, so stale contents of the first must not leak in)."""
import numpy as np
import pytest

import synth
from conftest import test_primes

pytestmark = pytest.mark.gpu


def test_noalloc_equals_det_mod_primes_twice_smaller_second():
    torch = pytest.importorskip("torch")
    import paper_cs_0511066_amd as det

    cases = [(300, 9, 81), (100, 4, 82)]                # second call smaller
    with det.Context(0) as ctx:
        for n, count, seed in cases:
            A = synth.dense_uniform(n, -1000, 1000, seed)
            A[:, 0] = 0
            A[n - 3, 0] = 7                              # a pivot from below (row swap)
            ps = test_primes(1 << 22, 1 << 23, count, seed) + test_primes(1 << 25, 1 << 26, 2, seed)
            At = torch.from_numpy(A).cuda()
            got = det.det_mod_primes_noalloc(At, ps)
            ref = ctx.det_mod_primes(At, ps, "fp64")
            print("noalloc n", n, "primes", len(ps), flush=True)
            assert got.tolist() == ref.tolist()


def test_noalloc_batches_and_stream():
    """n = 1024 with more primes than one batch of the 64 MiB array holds,
    on a caller's stream; then a small singular matrix (all residues 0)."""
    torch = pytest.importorskip("torch")
    import paper_cs_0511066_amd as det

    A = synth.dense_uniform(1024, 0, 255, 1024)
    ps = test_primes(1 << 22, 1 << 23, 20, 83)
    At = torch.from_numpy(A).cuda()
    s = torch.cuda.Stream()
    got = det.det_mod_primes_noalloc(At, ps, hip_stream=s.cuda_stream)
    with det.Context(0) as ctx:
        ref = ctx.det_mod_primes(At, ps, "fp64")
    assert got.tolist() == ref.tolist()
    S = synth.dense_uniform(40, -9, 9, 84)
    S[5] = S[6] - S[7]
    assert det.det_mod_primes_noalloc(torch.from_numpy(S).cuda(), ps[:3]).tolist() == [0, 0, 0]


def test_noalloc_rejects_what_it_cannot_do():
    torch = pytest.importorskip("torch")
    import paper_cs_0511066_amd as det

    ps = test_primes(1 << 22, 1 << 23, 2, 85)
    with pytest.raises(det.DetError) as e:                  # host memory: no staging without allocation
        det.det_mod_primes_noalloc(synth.dense_uniform(8, -5, 5, 1), ps)
    assert e.value.status == 1
    big = torch.full((16, 16), 2 ** 31, dtype=torch.int64, device="cuda")
    with pytest.raises(det.DetError) as e:
        det.det_mod_primes_noalloc(big, ps)
    assert e.value.status == 5
    with pytest.raises(det.DetError) as e:
        det.det_mod_primes_noalloc(torch.zeros((4096, 4096), dtype=torch.int64, device="cuda"), ps)
    assert e.value.status == 1
