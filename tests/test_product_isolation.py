"""The product path stands apart from the oracle and fails loudly without its
library (host checks, no GPU): no module of the package imports the oracle,
no HIP/C++ source includes it, the built library does not link it, and the
binding raises when libchem.so is missing instead of falling back."""
import ast
import os
import re
import subprocess
import sys

import pytest

from paper_2011_07978_amd import chem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2011_07978_amd")


def _py_modules():
    return sorted(os.path.join(PKG, f) for f in os.listdir(PKG) if f.endswith(".py"))


def test_package_sources_never_import_the_oracle():
    for path in _py_modules():
        tree = ast.parse(open(path).read(), path)
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            else:
                continue
            for n in names:
                assert n.split(".")[0] != "oracle", f"{path} imports {n}"
    csrc = os.path.join(PKG, "csrc")
    for f in sorted(os.listdir(csrc)):
        txt = open(os.path.join(csrc, f)).read()
        assert not re.search(r"#\s*include\s*[<\"][^>\"]*oracle", txt), f


def test_importing_the_package_loads_no_oracle():
    code = ("import sys\n"
            "import paper_2011_07978_amd.chem, paper_2011_07978_amd.synth\n"
            "import paper_2011_07978_amd.studies, paper_2011_07978_amd.accounting\n"
            "import paper_2011_07978_amd.surrogate\n"
            "assert not any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules), "
            "sorted(m for m in sys.modules if m.startswith('oracle'))\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]


def test_library_does_not_link_the_oracle():
    if not os.path.exists(chem.LIB_PATH):
        pytest.skip("libchem.so not built")
    r = subprocess.run(["readelf", "-d", chem.LIB_PATH], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("readelf not available")
    needed = re.findall(r"\(NEEDED\)\s+Shared library: \[([^\]]+)\]", r.stdout)
    assert needed, r.stdout[:500]
    assert not any("oracle" in n for n in needed), needed


def test_missing_library_raises():
    saved = chem._lib
    chem._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            chem.load_library(os.path.join(ROOT, "no_such_dir", "libchem.so"))
    finally:
        chem._lib = saved
