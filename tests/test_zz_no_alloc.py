"""kl_reduce_fp64_noalloc (the reduction entry point that allocates nothing)
against kl_reduce_fp64 through the C ABI: the same kernels on the same
inputs, so the FP64 sums, squares and maxima must agree bit for bit.  Two
calls in a row, the second on a smaller grid, check that the shared fixed
scratch carries nothing from one call into the next; the checksums of the
first call are also held to the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import Case, kl_mod as kl

pytestmark = pytest.mark.gpu


def _both(m, g, what, f, n):
    import torch
    a = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    b = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    m.kl_reduce_fp64(g, what, *f, a)
    m.kl_reduce_fp64_noalloc(g, what, *f, b)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_noalloc_reduction_equals_allocating_entry_point(dtype):
    m = kl()
    # a large grid on the 16-byte vector path, then a small ragged one on the
    # one-point-per-thread path
    for shape, seed in (((96, 40, 33), 5), ((21, 7, 5), 6)):
        c = Case(*shape, dtype, bc=0, seed=seed)
        for what, n in ((1, 9), (0, 3)):
            a, b = _both(m, c.g, what, c.dev, n)
            assert np.all(np.isfinite(b)), (shape, what, b)
            assert a.tobytes() == b.tobytes(), (shape, what, a, b)
        # the checksums against the oracle, as for kl_reduce_fp64
        a, b = _both(m, c.g, 1, c.dev, 9)
        for q, h in enumerate(c.host):
            ref = oracle.checksums(c.og, h)
            x = c.interior_np(h)
            assert abs(b[3 * q] - ref[0]) <= 1e-12 * np.sum(np.abs(x))
            assert abs(b[3 * q + 1] - ref[1]) <= 1e-12 * ref[1]
            assert b[3 * q + 2] == ref[2]


def test_noalloc_reduction_checks_arguments():
    m = kl()
    c = Case(8, 4, 3, 0, bc=0, seed=1)
    import torch
    out = torch.zeros(9, dtype=torch.float64, device="cuda")
    with pytest.raises(m.KLError):
        m.kl_reduce_fp64_noalloc(c.g, 7, *c.dev, out)
    with pytest.raises(m.KLError):
        m.kl_reduce_fp64_noalloc(c.g, 0, c.dev[0], None, c.dev[2], out)
