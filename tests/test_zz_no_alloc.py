"""mb_eval_direct_noalloc (no device allocation) against mb_eval_direct_unchecked.

Two calls in a row through the C ABI, the second on a smaller point set, so
the library's shared scratch array is reused with stale contents from the
first call; each result must equal the allocating entry point's on the same
points (same kernels: only the order of binary64 additions may differ).  Also
the size limit and argument errors.
"""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def run(fn_name, x, prec):
    import torch

    from paper_1105_2769_amd import _lib

    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    phi = torch.full((x.shape[0],), float("nan"), dtype=torch.float64, device="cuda:0")
    st = getattr(_lib.lib(), fn_name)(ctypes.c_void_p(xt.data_ptr()), x.shape[0],
                                      _lib.PREC[prec], ctypes.c_void_p(phi.data_ptr()),
                                      _lib.stream_of(xt))
    torch.cuda.synchronize()
    return st, phi.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_noalloc_equals_unchecked_two_calls(prec, cuda):
    for n, seed in ((1024, 71), (517, 72)):  # the second call is smaller
        x = workloads.jittered_lattice(n, seed=seed)
        print(f"noalloc {prec} n={n}", flush=True)
        st, got = run("mb_eval_direct_noalloc", x, prec)
        assert st == 0
        st, want = run("mb_eval_direct_unchecked", x, prec)
        assert st == 0
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=0.0)


def test_noalloc_limits(cuda):
    from paper_1105_2769_amd import _lib

    lib = _lib.lib()
    assert lib.mb_eval_direct_noalloc(None, 1025, 0, None, None) in (1, 5)
    x = workloads.jittered_lattice(1025, seed=1)
    st, _ = run("mb_eval_direct_noalloc", x, "fp64")
    assert st == 5  # MB_ERR_UNSUPPORTED above 1024 points
    assert lib.mb_eval_direct_noalloc(None, -1, 0, None, None) == 1
    assert lib.mb_eval_direct_noalloc(None, 0, 0, None, None) == 0
    for n in (1, 2):
        st, got = run("mb_eval_direct_noalloc", workloads.uniform_cube(n, 3), "fp64")
        assert st == 0 and np.all(got == 0.0)
