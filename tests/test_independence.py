"""The oracle and the product path share no code: no module of the package
imports the oracle, the oracle imports nothing of the package, and only
tests, the smoke check and the benchmark reach the oracle."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports(path):
    tree = ast.parse(open(path).read(), filename=path)
    out = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.level == 0 and node.module:
            out.add(node.module.split(".")[0])
    return out


def _py_files(d):
    for dirpath, _, files in os.walk(os.path.join(ROOT, d)):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(dirpath, f)


def test_package_does_not_import_the_oracle():
    bad = [p for p in _py_files("paper_2101_09059_amd") if "oracle" in _imports(p)]
    assert not bad, bad


def test_oracle_imports_nothing_of_the_package():
    bad = [p for p in _py_files("oracle") if "paper_2101_09059_amd" in _imports(p)]
    assert not bad, bad


def test_oracle_users_are_tests_smoke_and_bench():
    users = set()
    for f in os.listdir(ROOT):
        if f.endswith(".py") and "oracle" in _imports(os.path.join(ROOT, f)):
            users.add(f)
    assert users <= {"bench.py", "__graft_entry__.py"}, users
