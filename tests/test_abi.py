"""The C-ABI library loads and exports every entry point include/*.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:pd|pdm)_[a-z0-9_]+)\s*\(", text)))


def libraries():
    return {
        "pd.h": os.path.join(ROOT, "paper_2506_05362_amd", "libpd_mi355x.so"),
        "pd_mlp.h": os.path.join(ROOT, "paper_2506_05362_amd", "libpd_mlp.so"),
    }


@pytest.mark.parametrize("header", sorted(os.path.basename(h) for h in glob.glob(os.path.join(ROOT, "include", "*.h"))))
def test_library_exports_every_declared_symbol(header):
    lib_path = libraries()[header]
    if not os.path.exists(lib_path):
        from paper_2506_05362_amd import build
        build.build()
    L = ctypes.CDLL(lib_path)
    names = declared(os.path.join(ROOT, "include", header))
    assert names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_without_gpu():
    from paper_2506_05362_amd import pd
    L = pd.lib()
    assert L.pd_status_string(0) == b"ok"
    assert L.pd_status_string(-5) == b"instability flagged"
    assert L.pd_last_error(None) == b"null context"


def test_binding_refuses_missing_library(tmp_path):
    from paper_2506_05362_amd import pd
    with pytest.raises(RuntimeError):
        pd.load_library(str(tmp_path / "nope.so"))
