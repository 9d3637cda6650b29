"""The no-allocation overlap (qsv_overlap_noalloc) against qsv_overlap through
the C ABI: same kernels, same block count, so the four FP64 sums agree bit for
bit; two calls in a row, the second on a smaller state, in both dtypes."""

import numpy as np
import pytest

import oracle
from paper_2102_02957_amd import binding as B

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def rand_state(torch, n, seed, tdt):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.linalg.norm(v)
    return v, torch.from_numpy(v).to(tdt).cuda().contiguous()


@pytest.mark.parametrize("dt", [B.QSV_C128, B.QSV_C64])
def test_overlap_noalloc_matches_overlap(torch, dt):
    tdt = torch.complex128 if dt == B.QSV_C128 else torch.complex64
    ctx = B.Context(dt)
    for n, seed in ((22, 1), (9, 2)):       # second call: a smaller input
        a_h, a = rand_state(torch, n, seed, tdt)
        b_h, b = rand_state(torch, n, seed + 10, tdt)
        want = ctx.overlap(a, b, n).cpu().numpy()
        out = torch.full((4,), -7.0, dtype=torch.float64, device="cuda")
        ctx.overlap_noalloc(a, b, n, out)
        got = out.cpu().numpy()
        assert np.array_equal(got, want), (n, got, want)
        # and against the oracle's FP64 overlap of the same (rounded) inputs
        ah = a.cpu().numpy().astype(np.complex128)
        bh = b.cpu().numpy().astype(np.complex128)
        ov = oracle.overlap(ah, bh)
        assert abs(got[0] - ov.real) < 1e-12 and abs(got[1] - ov.imag) < 1e-12
        assert abs(got[2] - oracle.norm2(ah)) < 1e-12 and abs(got[3] - oracle.norm2(bh)) < 1e-12
