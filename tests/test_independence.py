"""The oracle and the product stay apart.  The HIP library and its binding
never import, include or run anything from oracle/, and the oracle never
imports the library.  The input generators (workloads.py) depend on neither.
Only tests/, bench.py's CPU-baseline leg and __graft_entry__.smoke() touch
the oracle."""
import ast
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2502_02395_amd")


def _imports(path):
    """(module, enclosing top-level function or None) for every import."""
    tree = ast.parse(open(path).read(), path)
    out = []

    def visit(node, fn):
        for ch in ast.iter_child_nodes(node):
            f = fn
            if isinstance(ch, (ast.FunctionDef, ast.AsyncFunctionDef)) and fn is None:
                f = ch.name
            if isinstance(ch, ast.Import):
                out.extend((a.name, f) for a in ch.names)
            elif isinstance(ch, ast.ImportFrom):
                out.append((ch.module or "", f))
            visit(ch, f)

    visit(tree, None)
    return out


def _top(mod):
    return mod.split(".")[0]


def test_product_does_not_use_the_oracle():
    py = glob.glob(os.path.join(PKG, "**", "*.py"), recursive=True)
    assert py
    for p in py:
        assert all("oracle" not in m.split(".") for m, _ in _imports(p)), p
    native = [p for e in ("cpp", "hip", "hpp", "h")
              for p in glob.glob(os.path.join(PKG, "csrc", "*." + e))]
    native += glob.glob(os.path.join(ROOT, "include", "*.h"))
    assert native
    for p in native:
        for inc in re.findall(r'#include\s*[<"]([^>"]+)[>"]', open(p).read()):
            assert "oracle" not in inc, (p, inc)


def test_oracle_does_not_use_the_product():
    for p in glob.glob(os.path.join(ROOT, "oracle", "*.py")):
        for m, _ in _imports(p):
            assert _top(m) not in ("paper_2502_02395_amd", "bench", "__graft_entry__"), (p, m)
            assert "csrc" not in m, (p, m)


def test_inputs_depend_on_neither():
    mods = {_top(m) for m, _ in _imports(os.path.join(ROOT, "workloads.py"))}
    assert not mods & {"oracle", "paper_2502_02395_amd", "torch"}, mods


def test_oracle_entry_points_outside_tests():
    for name, allowed in (("bench.py", {"cpu_baseline"}), ("__graft_entry__.py", {"smoke"})):
        uses = [(m, f) for m, f in _imports(os.path.join(ROOT, name)) if _top(m) == "oracle"]
        assert uses, name
        assert {f for _, f in uses} <= allowed, (name, uses)
