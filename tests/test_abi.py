"""The C-ABI library builds, loads and exports every entry point that
include/lbib.h declares; host-side validation works without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbib.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbib_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1906_03065_amd import lbib

    L = lbib.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    bound = {s[0] for s in lbib.SIGNATURES}
    assert set(names) == bound


def test_workspace_and_validation_on_host():
    from paper_1906_03065_amd import lbib
    from paper_1906_03065_amd import workloads as W

    w = W.c1()
    prm = lbib.make_params(w["params"], "fp32", membranes=w["membranes"])
    n32 = lbib.workspace_bytes(prm)
    prm64 = lbib.make_params(w["params"], "fp64", membranes=w["membranes"])
    assert lbib.workspace_bytes(prm64) > n32 > 2 * 128 * 128 * 27 * 4
    bad = lbib.make_params(dict(w["params"], tau=0.5), "fp32")
    with pytest.raises(lbib.LbibError):
        lbib.workspace_bytes(bad)
    bad = lbib.make_params(dict(w["params"], nz=2), "fp32")
    with pytest.raises(lbib.LbibError):
        lbib.workspace_bytes(bad)
    assert lbib.lib().lbib_strerror(-1) == b"invalid argument"
