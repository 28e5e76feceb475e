"""The oracle and the HIP path share no code: no module of the package imports
the oracle, the oracle imports nothing of the package, and outside the test
suite only the smoke check and the benchmark's CPU-baseline leg load it.
Checked on the source text (import statements), so it needs no GPU."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = "paper_1701_08361_amd"


def _imports(path):
    """(module name, name of the enclosing function or None) of every import."""
    tree = ast.parse(open(path, encoding="utf-8").read())
    out = []

    def visit(node, func):
        for child in ast.iter_child_nodes(node):
            f = child.name if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) else func
            if isinstance(child, ast.Import):
                out.extend((a.name, func) for a in child.names)
            elif isinstance(child, ast.ImportFrom):
                mod = ("." * child.level) + (child.module or "")
                out.append((mod, func))
            visit(child, f)

    visit(tree, None)
    return out


def _py_files(d):
    for base, _, files in os.walk(os.path.join(ROOT, d)):
        if "__pycache__" in base:
            continue
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(base, f)


def test_package_never_imports_the_oracle():
    for path in _py_files(PKG):
        for mod, _ in _imports(path):
            assert not mod.split(".")[0] == "oracle", f"{path} imports {mod}"


def test_oracle_imports_nothing_of_the_package():
    for path in _py_files("oracle"):
        for mod, _ in _imports(path):
            assert mod.split(".")[0] not in (PKG, ""), f"{path} imports {mod}"


def test_oracle_users_outside_the_tests():
    users = {}
    for path in [os.path.join(ROOT, "bench.py"), os.path.join(ROOT, "__graft_entry__.py")]:
        users[os.path.basename(path)] = {f for mod, f in _imports(path) if mod.split(".")[0] == "oracle"}
    assert users["bench.py"] == {"cpu_baseline"}
    assert users["__graft_entry__.py"] == {"smoke"}


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No fallback: without libnlinv.so every plan fails at load time."""
    import pytest
    from paper_1701_08361_amd import nlinv as nl
    monkeypatch.setattr(nl, "_lib", None)
    monkeypatch.setattr(nl, "LIB_PATH", str(tmp_path / "missing" / "libnlinv.so"))
    with pytest.raises(FileNotFoundError):
        nl.load()
    with pytest.raises(FileNotFoundError):
        nl.make_params(64, 8, 13)
