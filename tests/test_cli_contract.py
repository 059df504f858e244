"""The command-line contracts that need no GPU: bench.py refuses more than one
GPU and a machine without one with a message (exit 2, no JSON line), the
build / smoke entry points exist, and smoke() refuses to run without a GPU
(no CPU fallback)."""
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def _run(*args):
    return subprocess.run([sys.executable, *args], cwd=ROOT, capture_output=True, text=True, timeout=300)


def test_bench_refuses_more_than_one_gpu():
    r = _run("bench.py", "--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_bench_needs_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = _run("bench.py", "--steps", "1")
    assert r.returncode == 2
    assert "needs a GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_entry_points_and_smoke_without_gpu():
    import torch
    sys.path.insert(0, str(ROOT))
    import __graft_entry__ as g
    assert callable(g.build) and callable(g.smoke)
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        g.smoke()


def test_stepbench_cli_parses():
    r = _run("-m", "paper_1205_6872_amd.stepbench", "--help")
    assert r.returncode == 0
    assert "--mirror" in r.stdout and "--paper-table1" in r.stdout


@pytest.mark.parametrize("warmup,F,want", [(5, 3, 7), (7, 3, 7), (0, 3, 1), (1, 3, 1), (5, 2, 5),
                                            (4, 2, 5), (5, 1, 5), (0, 1, 1)])
def test_bench_warmup_starts_the_timed_call_on_a_group(warmup, F, want):
    # groups start at n = L+1, L+1+F, ...; the timed call starts at step L + W
    sys.path.insert(0, str(ROOT))
    import bench
    w = bench.aligned_warmup(warmup, F)
    assert w == want
    L = 15
    assert (L + w - L - 1) % F == 0 and w >= max(1, warmup)
