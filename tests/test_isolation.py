"""The product path and the oracle share nothing: no module of the package
imports the oracle, no library source includes or names its header or
library, and the built library does not link it."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2006_13631_amd")


def _files(exts):
    for d, _, fs in os.walk(PKG):
        if "__pycache__" in d:
            continue
        for f in fs:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_package_modules_do_not_import_the_oracle():
    pat = re.compile(r"^\s*(from\s+oracle\b|import\s+oracle\b|from\s+\.\.?oracle\b)", re.M)
    bad = [p for p in _files((".py",)) if pat.search(open(p).read())]
    assert not bad, bad


def test_library_sources_do_not_name_the_oracle():
    pat = re.compile(r"hlbm_oracle|liboracle|\bor_(create|step|set_threads)\b")
    bad = [p for p in _files((".hip", ".h", ".cpp")) if pat.search(open(p).read())]
    assert not bad, bad
    for h in os.listdir(os.path.join(ROOT, "include")):
        assert not pat.search(open(os.path.join(ROOT, "include", h)).read()), h


def test_built_library_does_not_link_the_oracle():
    lib = os.path.join(PKG, "libhlbm.so")
    if not os.path.exists(lib):
        import pytest
        pytest.skip("library not built")
    out = subprocess.run(["readelf", "-d", lib], capture_output=True, text=True).stdout
    needed = re.findall(r"\(NEEDED\).*\[(.*)\]", out)
    assert needed and not [n for n in needed if "oracle" in n], needed
