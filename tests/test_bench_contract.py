"""CPU checks of bench.py: every --workload choice dispatches to a function
that exists, and more than one GPU is refused with a message."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_every_workload_has_a_function():
    tree = ast.parse(open(BENCH).read())
    defs = {n.name for n in tree.body if isinstance(n, ast.FunctionDef)}
    choices, called = None, set()
    for node in ast.walk(tree):
        if isinstance(node, ast.keyword) and node.arg == "choices":
            choices = [e.value for e in node.value.elts]
        if isinstance(node, ast.Call) and isinstance(node.func, ast.Name) and \
                node.func.id.startswith("run_"):
            called.add(node.func.id)
    assert choices and "product" in choices
    for name in called:
        assert name in defs, name
    for w in choices:
        if w != "product":
            assert "run_" + w in defs, w


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
