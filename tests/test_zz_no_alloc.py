"""mj_kernel_values_noalloc (staging through the library's fixed device array) against
mj_kernel_values (staging buffers allocated per call), through the C-ABI."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _requests(rng, n, U, V, W, ell):
    lags = rng.integers(0, ell + 1, n).astype(np.int32)
    offs = np.stack([rng.integers(-(U - 1), U, n), rng.integers(-(V - 1), V, n),
                     rng.integers(-(W - 1), W, n)], axis=1).astype(np.int32)
    return lags, offs


def test_kernel_values_noalloc_matches_allocating_call():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_03323_amd import build, solver_for
    from paper_2407_03323_amd.motjvie import MJ_EINVAL, MotJvieError
    assert build.is_current()
    U, V, W = 7, 5, 6
    prob = wl.Problem("na", U, V, W, wl.random_eps(U, V, W, 3, 2.0, 9.0), [], 1)
    s = solver_for(prob)
    ell = s.ell
    rng = np.random.default_rng(2024)
    # two calls in a row, the second smaller: the staging array keeps the first call's values
    # beyond the second's requests, which must not leak into its results
    for n in (4000, 137):
        lags, offs = _requests(rng, n, U, V, W, ell)
        ref = s.kernel_values(lags, offs)
        got = s.kernel_values_noalloc(lags, offs)
        print("noalloc n=%d max|diff| %.3g" % (n, np.abs(got - ref).max()), flush=True)
        assert got.shape == (n, 6)
        assert np.array_equal(got, ref)
    assert s.kernel_values_noalloc(np.zeros(0, np.int32), np.zeros((0, 3), np.int32)).shape == (0, 6)
    # host-side limits: more requests than the array holds, a lag or an offset out of range
    with pytest.raises(MotJvieError) as ei:
        s.kernel_values_noalloc(np.zeros(65537, np.int32), np.zeros((65537, 3), np.int32))
    assert ei.value.code == MJ_EINVAL
    with pytest.raises(MotJvieError) as ei:
        s.kernel_values_noalloc([ell + 1], [[0, 0, 0]])
    assert ei.value.code == MJ_EINVAL
    with pytest.raises(MotJvieError) as ei:
        s.kernel_values_noalloc([1], [[U, 0, 0]])
    assert ei.value.code == MJ_EINVAL
    s.close()
