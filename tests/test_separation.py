"""The oracle and the HIP path share no code, and the oracle is reached only from the places
allowed to use it: the tests, the smoke check and the benchmark's CPU-baseline leg."""
import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2111_05205_amd")


def _files(top, exts):
    for d, _, names in os.walk(top):
        if "__pycache__" in d or "_build" in d:
            continue
        for n in names:
            if n.endswith(exts):
                yield os.path.join(d, n)


def _oracle_imports(path):
    """(enclosing function or '<module>', line) of every import of the oracle package."""
    tree = ast.parse(open(path).read())
    found = []

    def visit(node, scope):
        for child in ast.iter_child_nodes(node):
            s = child.name if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) else scope
            if isinstance(child, ast.ImportFrom) and (child.module or "").split(".")[0] == "oracle":
                found.append((scope, child.lineno))
            elif isinstance(child, ast.Import) and any(a.name.split(".")[0] == "oracle" for a in child.names):
                found.append((scope, child.lineno))
            visit(child, s)
    visit(tree, "<module>")
    return found


def test_package_never_reaches_the_oracle():
    for path in _files(PKG, (".py",)):
        assert not _oracle_imports(path), path
    for path in _files(os.path.join(PKG, "csrc"), (".hip", ".h", ".cpp")):
        assert not re.search(r"oracle", open(path).read(), re.I), path
    for path in _files(os.path.join(ROOT, "include"), (".h",)):
        assert "oracle" not in open(path).read().lower(), path


def test_oracle_never_reaches_the_package():
    for path in _files(os.path.join(ROOT, "oracle"), (".py", ".c", ".h")):
        src = open(path).read()
        assert "paper_2111_05205_amd" not in src and "tdbem" not in src, path


def test_benchmark_and_entry_use_the_oracle_only_where_allowed():
    assert {s for s, _ in _oracle_imports(os.path.join(ROOT, "bench.py"))} <= {"cpu_baseline"}
    assert {s for s, _ in _oracle_imports(os.path.join(ROOT, "__graft_entry__.py"))} <= {"build", "smoke"}
