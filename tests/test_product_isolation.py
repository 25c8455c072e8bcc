"""The product path stands alone: it never reaches the oracle, and it fails
loudly, with no CPU fallback, when the HIP library is missing."""
import glob
import os
import re

import pytest

from conftest import ROOT
from paper_1809_09851_amd import fdbb as F

PKG = os.path.join(ROOT, "paper_1809_09851_amd")


def test_product_sources_do_not_reference_the_oracle():
    sources = glob.glob(os.path.join(PKG, "*.py")) + glob.glob(os.path.join(PKG, "csrc", "*"))
    sources += glob.glob(os.path.join(ROOT, "include", "*.h"))
    assert len(sources) > 15
    for path in sources:
        text = open(path, errors="replace").read()
        assert not re.search(r"\boracle\b", text, re.I), path


def test_missing_library_raises(monkeypatch):
    monkeypatch.setattr(F, "LIBRARY", os.path.join(ROOT, "no_such_dir", "libfdbb.so"))
    monkeypatch.setattr(F, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        F.library()
    with pytest.raises(RuntimeError, match="not built"):
        F.fdbb_get_launch_config("flux", 3, F.F64)
