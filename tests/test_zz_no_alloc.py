"""pod_center_rows_noalloc (no device allocation, the library's device
scratch) against pod_center_rows (scratch allocated per call): bit for bit,
on two calls in a row, the second with a smaller input, in FP32 and FP64;
sizes beyond the scratch are refused before anything runs."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1905_05107_amd as pod  # noqa: E402


def _case(m, n, dtype, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, m)) + 5.0 * rng.standard_normal((1, m))   # row offsets to remove
    return torch.from_numpy(A.astype(dtype)).cuda()                       # (n, m): A = t.T, column-major


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_center_rows_noalloc_equals_the_allocating_call(dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for m, n, seed in [(300_007, 70, 1), (9_001, 33, 2)]:       # the second call is smaller
        print(f"noalloc centring m={m} n={n} {dtype.__name__}", flush=True)
        t = _case(m, n, dtype, seed)
        want = t.clone()
        got = t.clone()
        pod.center_rows(want.T)
        st = torch.cuda.current_stream()
        rc = pod.lib().pod_center_rows_noalloc(ctypes.c_void_p(got.data_ptr()), pod.POD_F64 if dtype == np.float64
                                               else pod.POD_F32, m, n, m, ctypes.c_void_p(st.cuda_stream))
        assert rc == pod.POD_OK
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        assert float(got.to(torch.float64).mean(dim=0).abs().max()) < 1e-5


def test_center_rows_noalloc_refuses_sizes_beyond_its_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    small = torch.zeros(16, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    m = (1 << 23) + 1      # one range of 2^23 + 1 doubles: more than the scratch holds
    rc = pod.lib().pod_center_rows_noalloc(ctypes.c_void_p(small.data_ptr()), pod.POD_F32, m, 1, m,
                                           ctypes.c_void_p(st.cuda_stream))
    assert rc == pod.POD_EINVAL
