"""CPU checks of the HIP library: it builds, loads, and exports every symbol
declared in include/hm.h (no compute calls here; those need the GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hm_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    from paper_1703_09085_amd import hm

    assert declared_symbols() == sorted(hm.SYMBOLS)


def test_library_exports_declared_symbols():
    from paper_1703_09085_amd import hm

    if not os.path.exists(hm.LIB_PATH):
        pytest.skip("libhm.so not built")
    lib = hm.lib()
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing
    assert lib.hm_version().decode().startswith("hm-gfx950")


def test_no_cpu_fallback_in_binding():
    """The binding never imports the oracle: the product path is GPU-only."""
    src = open(os.path.join(ROOT, "paper_1703_09085_amd", "hm.py")).read()
    assert "oracle" not in src.replace("no CPU fallback", "")
