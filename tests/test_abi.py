"""CPU-side checks of the C ABI: the library loads, exports every entry point
declared in include/pod.h, and its host-only helpers agree with the paper's
formulas as the oracle states them.  No device work is launched here."""
import os
import re

import pytest

import paper_1905_05107_amd as pod
from oracle.isma import sample_size_ctsvd, sample_size_ltsvd

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


@pytest.mark.parametrize("k,eps,delta", [(10, 0.7, 0.6), (2, 0.7, 0.6), (20, 0.6, 0.6), (5, 0.6, 0.6), (10, 1.0, 0.75)])
def test_sample_size_helpers(k, eps, delta):
    if not os.path.exists(pod.LIB_PATH):
        pytest.skip("libpod.so not built")
    assert pod.sample_size("ltsvd", k, eps, delta) == sample_size_ltsvd(k, eps, delta)
    assert pod.sample_size("ctsvd", k, eps, delta) == sample_size_ctsvd(k, eps, delta)


def test_status_strings():
    if not os.path.exists(pod.LIB_PATH):
        pytest.skip("libpod.so not built")
    assert pod.status_str(pod.POD_OK) == "ok"
    assert "sample" in pod.status_str(pod.POD_EXHAUSTED)
