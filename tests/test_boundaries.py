"""Static checks of the separation between the product and the oracle:
the package never references the oracle, and bench.py imports it only in
its CPU-baseline leg."""
import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_package_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2206_06302_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f), errors="ignore").read()
                assert not re.search(r"\bimport\s+oracle\b|\bfrom\s+oracle\b|oracle\.h|liboracle", text), f


def test_bench_uses_the_oracle_only_in_the_cpu_baseline_leg():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    for fn in [n for n in ast.walk(tree) if isinstance(n, ast.FunctionDef)]:
        for node in ast.walk(fn):
            names = []
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            if any(n.split(".")[0] == "oracle" for n in names):
                assert fn.name == "cpu_baseline_leg", fn.name
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))]
    for node in top:
        names = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
        assert not any(n.split(".")[0] == "oracle" for n in names)


def test_oracle_and_product_share_no_source():
    ora = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert "ts_device" not in ora and "tstream" not in ora
