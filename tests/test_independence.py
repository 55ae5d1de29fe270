"""The oracle and the HIP path share no code: the HIP sources include only
their own headers, the public headers and system headers; no product module
imports the oracle; the oracle includes only its own header and the C
library, and imports nothing from the package; the seeded input generators
import neither side.  CPU only."""
import ast
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1806_08741_amd")
CSRC = os.path.join(PKG, "csrc")
ORACLE = os.path.join(ROOT, "oracle")


def includes(path):
    with open(path, encoding="utf-8") as fh:
        return re.findall(r'^\s*#\s*include\s*([<"])([^>"]+)[>"]', fh.read(), re.M)


def imports(path):
    with open(path, encoding="utf-8") as fh:
        tree = ast.parse(fh.read())
    out = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.module:
            out.add(node.module.split(".")[0])
    return out


def test_hip_sources_include_only_their_own_and_public_headers():
    own = {os.path.basename(p) for p in glob.glob(os.path.join(CSRC, "*.h"))}
    public = {os.path.basename(p) for p in glob.glob(os.path.join(ROOT, "include", "*.h"))}
    for src in glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h")):
        for kind, name in includes(src):
            if kind == "<":
                assert "oracle" not in name, (src, name)
                continue
            base = os.path.basename(name)
            assert "oracle" not in name, (src, name)
            assert base in own or (base in public and "include/" in name), (src, name)


def test_oracle_includes_only_itself_and_the_c_library():
    for src in glob.glob(os.path.join(ORACLE, "*.c")) + glob.glob(os.path.join(ORACLE, "*.h")):
        for kind, name in includes(src):
            if kind == '"':
                assert name == "sslic_oracle.h", (src, name)
            else:
                assert not name.startswith(("hip", "sslic")), (src, name)


def test_product_modules_do_not_import_the_oracle():
    for mod in glob.glob(os.path.join(PKG, "*.py")):
        assert "oracle" not in imports(mod), mod


def test_oracle_and_generators_import_neither_side():
    for mod in glob.glob(os.path.join(ORACLE, "*.py")):
        assert "paper_1806_08741_amd" not in imports(mod), mod
    assert not imports(os.path.join(PKG, "synth.py")) & {"oracle", "paper_1806_08741_amd"}
    with open(os.path.join(PKG, "synth.py"), encoding="utf-8") as fh:
        text = fh.read()
    assert "from . import sslic" not in text and "import sslic" not in text
