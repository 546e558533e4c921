"""The product path and the oracle share no code: neither imports the
other, and importing the product does not load the oracle."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2401_11324_amd")
ORACLE = os.path.join(ROOT, "oracle")


def sources(d, exts):
    for dp, _, fs in os.walk(d):
        for f in fs:
            if f.endswith(exts):
                yield os.path.join(dp, f)


def test_product_sources_do_not_reference_the_oracle():
    for p in sources(PKG, (".py", ".hip", ".cpp", ".h")):
        txt = open(p).read()
        assert not re.search(r"\boracle\b", txt), p
        assert "_oracle.so" not in txt, p


def test_oracle_sources_do_not_reference_the_product():
    for p in sources(ORACLE, (".py", ".c", ".h")):
        txt = open(p).read()
        assert "paper_2401_11324_amd" not in txt, p
        assert "bang_kernels" not in txt and "bang.h" not in txt, p


def test_importing_the_product_loads_no_oracle_module():
    code = ("import sys; sys.path.insert(0, %r); import paper_2401_11324_amd;"
            "paper_2401_11324_amd.lib();"
            "print(any(m == 'oracle' or m.startswith('oracle.') "
            "for m in sys.modules))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True,
                         text=True, check=True)
    assert out.stdout.strip() == "False"
