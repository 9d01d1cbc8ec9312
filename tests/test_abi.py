"""CPU-side checks of the C ABI: the library loads, exports every entry point
declared in include/pod.h, and its host-only helpers agree with the paper's
formulas (hand-derived values).  No device work is launched here."""
import os
import re

import pytest

import paper_1905_05107_amd as pod
from test_oracle_pins_sampling import CTSVD_TABLE, LTSVD_TABLE

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pod_[a-z_0-9]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(pod.LIB_PATH):
        pytest.skip("libpod.so not built")
    L = pod.lib()
    declared = _declared()
    assert declared, "no declarations found"
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert set(pod.EXPORTS) == declared


@pytest.mark.parametrize("args,want", LTSVD_TABLE)
def test_sample_size_ltsvd_hand_derived(args, want):
    if not os.path.exists(pod.LIB_PATH):
        pytest.skip("libpod.so not built")
    assert pod.sample_size("ltsvd", *args) == want


@pytest.mark.parametrize("args,want", CTSVD_TABLE)
def test_sample_size_ctsvd_hand_derived(args, want):
    if not os.path.exists(pod.LIB_PATH):
        pytest.skip("libpod.so not built")
    assert pod.sample_size("ctsvd", *args) == want


def test_sample_size_rejects_invalid_arguments():
    if not os.path.exists(pod.LIB_PATH):
        pytest.skip("libpod.so not built")
    for kind, k, eps, delta in [("ltsvd", 0, 0.5, 0.5), ("ltsvd", 3, 0.0, 0.5), ("ltsvd", 3, 0.5, 1.0),
                                ("ctsvd", 3, 0.5, 2.0), ("ctsvd", 3, -1.0, 0.5)]:
        assert pod.sample_size(kind, k, eps, delta) == -1


def test_status_strings():
    if not os.path.exists(pod.LIB_PATH):
        pytest.skip("libpod.so not built")
    assert pod.status_str(pod.POD_OK) == "ok"
    assert "sample" in pod.status_str(pod.POD_EXHAUSTED)


def test_wedin_inputs_are_checked_before_the_call():
    """The quality-measure kernels read k columns of m (U) and n (V) rows in
    the output type; wrong shapes, dtypes, devices or layouts are refused on
    the host (CPU tensors stand in for the device here)."""
    torch = pytest.importorskip("torch")
    m, n, k = 7, 5, 3
    dev = torch.device("cpu")
    U = torch.zeros((k, m), dtype=torch.float32).T
    V = torch.zeros((k, n), dtype=torch.float32).T
    pod.check_pairs(U, V, m, n, k, torch.float32, dev)
    bad = [
        (torch.zeros((k - 1, m), dtype=torch.float32).T, V, torch.float32),   # fewer columns
        (U, torch.zeros((k, n + 1), dtype=torch.float32).T, torch.float32),   # wrong rows
        (U, V, torch.float64),                                                 # FP32 pairs on an FP64 context
        (torch.zeros((m, k), dtype=torch.float32), V, torch.float32),          # row-major U
    ]
    for Ub, Vb, dt in bad:
        with pytest.raises(ValueError):
            pod.check_pairs(Ub, Vb, m, n, k, dt, dev)
    with pytest.raises(ValueError):
        pod.check_pairs(U, V, m, n, k, torch.float32, torch.device("cuda", 0))  # host tensors


def test_stop_reason_names_cover_the_enum():
    txt = open(os.path.join(ROOT, "include", "pod.h")).read()
    codes = dict((name, int(v)) for name, v in re.findall(r"\b(POD_STOP_[A-Z_]+)\s*=\s*(\d+)", txt))
    assert codes == {"POD_STOP_NONE": pod.POD_STOP_NONE, "POD_STOP_NONFINITE": pod.POD_STOP_NONFINITE,
                     "POD_STOP_CONVERGED": pod.POD_STOP_CONVERGED, "POD_STOP_EXHAUSTED": pod.POD_STOP_EXHAUSTED,
                     "POD_STOP_MAX_ITER": pod.POD_STOP_MAX_ITER, "POD_STOP_BREAKDOWN": pod.POD_STOP_BREAKDOWN}
    assert set(pod.STOP_NAMES) == set(codes.values())
