"""Static checks of bench.py and __graft_entry__.py on the CPU: every name
they call is defined, imported or a builtin (a missing helper would only
show up on a GPU run), and the multi-GPU request exits with its message."""
import ast
import builtins
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _undefined_calls(path):
    tree = ast.parse(open(path).read())
    known = set(dir(builtins))
    for node in ast.walk(tree):
        if isinstance(node, (ast.FunctionDef, ast.ClassDef)):
            known.add(node.name)
            known.update(a.arg for a in node.args.args + node.args.kwonlyargs) if isinstance(node, ast.FunctionDef) else None
        elif isinstance(node, (ast.Import, ast.ImportFrom)):
            known.update((a.asname or a.name).split(".")[0] for a in node.names)
        elif isinstance(node, ast.Name) and isinstance(node.ctx, ast.Store):
            known.add(node.id)
        elif isinstance(node, ast.arg):
            known.add(node.arg)
        elif isinstance(node, (ast.comprehension,)):
            for n in ast.walk(node.target):
                if isinstance(n, ast.Name):
                    known.add(n.id)
    missing = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Call) and isinstance(node.func, ast.Name) and node.func.id not in known:
            missing.add(node.func.id)
    return missing


@pytest.mark.parametrize("name", ["bench.py", "__graft_entry__.py"])
def test_every_called_name_is_defined(name):
    assert _undefined_calls(os.path.join(ROOT, name)) == set()


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_roofline_kernel_names_match_the_profiles():
    """The roofline's kernel name is the one the rocprofv3 summaries are keyed
    by (template instantiation included), and its source file is the one that
    defines it, so the traffic lookup can find the counters."""
    sys.path.insert(0, ROOT)
    import json
    import bench
    assert bench.scan_kernels([50, 70] * 4) == ["k_scanlines<2, 0>"]   # n = 51, 71
    assert bench.scan_kernels([32]) == ["k_scanlines<2, 0>"]           # n = 33
    assert bench.scan_kernels([200, 400]) == ["k_scanlines<4, 0>", "k_scanlines<8, 0>"]
    assert bench.scan_kernels([1023]) == ["k_scanlines<16, 0>"]
    keys = set(json.load(open(os.path.join(ROOT, "profiles", "traffic.json"))))
    kernels = {k.split(" @ ")[0] for k in keys - {"copy_probe"}}
    assert {"k_scanlines<2, 0>", "k_edges", "k_scanlines_batched<2, 0>"} <= kernels
    assert bench.traffic_key("k_scanlines_batched<2, 0>", bench.BATCH_WORKLOAD) in keys
    for k in kernels:
        base = k.split("<")[0]
        src = open(os.path.join(ROOT, bench.kernel_source(k))).read()
        assert f"void {base}(" in src or f"void {base}\n" in src or f" {base}(" in src, (k, bench.kernel_source(k))
