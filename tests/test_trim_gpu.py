"""mb_trim: the library's cached device memory goes back to the device, and
later calls allocate again and give the same results."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_trim_releases_pool_memory(cuda):
    import torch

    import paper_1105_2769_amd as mb

    n = 8192
    x = torch.from_numpy(workloads.jittered_lattice(n, seed=3)).to(cuda)
    print("trim: exhaustive sum, then trim", flush=True)
    first = mb.eval_direct_deterministic(x).cpu().numpy()
    # the binary64 (i, j) table of 128 x 128 blocks of 64 x 64 pairs, 16 bytes
    # a pair, went back to the pool when the call ended
    table = (n // 64) ** 2 * 64 * 64 * 16
    released = mb.trim()
    print(f"trim released {released} bytes", flush=True)
    assert released >= table
    assert mb.trim() == 0
    again = mb.eval_direct_deterministic(x).cpu().numpy()
    assert np.array_equal(first.view(np.uint64), again.view(np.uint64))
