"""Host checks of bench.py that need no GPU: every name it reads is bound somewhere
(a function lost in an edit fails here instead of after minutes of GPU work), and
its argument parsing and helpers behave."""
import ast
import builtins
import pathlib

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]


def _bound_names(tree):
    names = set(dir(builtins)) | {"__file__", "__name__", "__doc__"}
    for node in ast.walk(tree):
        if isinstance(node, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            names.add(node.name)
        elif isinstance(node, ast.Name) and isinstance(node.ctx, (ast.Store, ast.Del)):
            names.add(node.id)
        elif isinstance(node, ast.arg):
            names.add(node.arg)
        elif isinstance(node, (ast.Import, ast.ImportFrom)):
            for a in node.names:
                names.add((a.asname or a.name).split(".")[0])
        elif isinstance(node, ast.ExceptHandler) and node.name:
            names.add(node.name)
    return names


@pytest.mark.parametrize("script", ["bench.py", "__graft_entry__.py"])
def test_every_name_read_is_bound(script):
    tree = ast.parse((ROOT / script).read_text())
    bound = _bound_names(tree)
    unbound = sorted({n.id for n in ast.walk(tree)
                      if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load) and n.id not in bound})
    assert not unbound, f"{script} reads names bound nowhere: {unbound}"


def test_full_trajectory_bytes_sums_rounded_streams():
    import bench
    st = {"profile": [1000.0] * 17}
    assert bench.full_trajectory_bytes(st, 10) == 10 * 1024.0


def test_raw_gpts_counts_every_stencil_update_over_kernel_time():
    import bench
    stats = [{"advances": 8442, "reverses": 3000, "ms_fwd_kernel": 8442 * 0.2, "ms_adj_kernel": 3000 * 0.4}] * 2
    # 11442 updates of 1e6 points in 2888.4 ms, twice
    assert bench.raw_gpts(stats, 1_000_000) == pytest.approx(11442e6 / 2.8884 / 1e9, abs=1e-3)
    assert bench.raw_gpts([{"advances": 1, "reverses": 1, "ms_fwd_kernel": 0.0, "ms_adj_kernel": 0.0}], 10) is None
