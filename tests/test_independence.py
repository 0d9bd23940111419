"""The oracle and the GPU library share no code: no source of the package
names the oracle, and the oracle's C file includes only the C standard
library (CPU only)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1712_06326_amd")


def _sources(top, exts):
    for d, _, files in os.walk(top):
        if "_build" in d or "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_package_never_names_the_oracle():
    for p in _sources(PKG, (".py", ".hip", ".cpp", ".hpp", ".h")):
        src = open(p, encoding="utf-8").read()
        assert not re.search(r"^\s*(import|from)\s+oracle\b", src, re.M), p
        assert not re.search(r"#\s*include\s*[<\"][^>\"]*oracle", src), p
        assert "liboracle" not in src, p


def test_oracle_includes_only_the_c_library():
    src = open(os.path.join(ROOT, "oracle", "oracle.c"), encoding="utf-8").read()
    heads = re.findall(r"#\s*include\s*([<\"][^>\"]+[>\"])", src)
    allowed = {"<math.h>", "<stdint.h>", "<stdlib.h>", "<string.h>", "<stdio.h>", "<stddef.h>",
               "<limits.h>", "<float.h>"}
    assert heads and set(heads) <= allowed, heads
