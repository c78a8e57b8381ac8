"""The oracle and the HIP path share no code: neither imports the other (no GPU)."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports(path):
    out = set()
    for dirpath, _, files in os.walk(path):
        for f in files:
            if f.endswith(".py"):
                tree = ast.parse(open(os.path.join(dirpath, f)).read())
                for node in ast.walk(tree):
                    if isinstance(node, ast.Import):
                        out.update(a.name.split(".")[0] for a in node.names)
                    elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
                        out.add(node.module.split(".")[0])
    return out


def test_oracle_does_not_import_product():
    assert "paper_2603_16850_amd" not in _imports(os.path.join(ROOT, "oracle"))


def test_product_does_not_import_oracle():
    assert "oracle" not in _imports(os.path.join(ROOT, "paper_2603_16850_amd"))


def test_product_sources_do_not_reference_oracle():
    for dirpath, _, files in os.walk(os.path.join(ROOT, "paper_2603_16850_amd")):
        for f in files:
            if f.endswith((".hip", ".cpp", ".h", ".hpp")):
                assert "oracle" not in open(os.path.join(dirpath, f)).read(), f
