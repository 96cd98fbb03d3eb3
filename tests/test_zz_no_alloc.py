"""The dot product entry point that allocates nothing (for callers under
graph capture or that forbid device allocation) against msp_vec_dot, the
allocating entry point it varies: the same kernel and grid, so the two
results must be bitwise equal.  Two calls in a row, the second with a
smaller input, check that the shared device scratch (partials and ticket
counter) carries nothing from one call into the next."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _msp():
    import paper_2006_13387_amd as msp
    msp.load_library()
    return msp


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def test_noalloc_dot_matches_allocating_dot_twice():
    msp = _msp()
    from paper_2006_13387_amd import binding
    rng = np.random.default_rng(77)
    # the first call fills all 1,024 partial slots, the second only a few
    for n in (5_000_003, 3_001):
        x, y = rng.standard_normal(n), rng.standard_normal(n)
        xd, yd = _dev(x), _dev(y)
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        print(f"[noalloc dot] n={n}", flush=True)
        binding.vec_dot_noalloc(xd, yd, out)
        torch.cuda.synchronize()
        got = float(out.cpu()[0])
        ref = msp.vec_dot(xd, yd)
        assert got == ref, (n, got, ref)
        assert abs(got - x @ y) <= 1e-12 * np.abs(x * y).sum()


def test_noalloc_dot_rejects_bad_sizes():
    L = _msp().load_library()
    from paper_2006_13387_amd import binding
    x = _dev(np.ones(4))
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(x.data_ptr())
    o = ctypes.c_void_p(out.data_ptr())
    assert L.msp_vec_dot_noalloc(-1, p, p, o, None) == -1
    assert L.msp_vec_dot_noalloc((1 << 35) + 1, p, p, o, None) == -1
    assert b"MAX_N" in L.msp_last_error(None)
    assert L.msp_vec_dot_noalloc(4, p, p, None, None) == -1
