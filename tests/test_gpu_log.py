"""GPU test of FEMH_LOG: a child process solves a small box with the
variable set (level 2) and once without it; the logged lines name the
problem, the solve's mode, each chunk's recursive residual (iteration
counts that do not decrease, ending at the reported count), the true
residual check and the final status, and nothing is logged by default."""
import os
import re
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import torch
assert torch.cuda.is_available()
import workloads as W
from paper_0704_2344_amd import femh as F
ctx = F.Context(0)
prob, waves = W.free_cube(5)
P = F.Problem(ctx, prob)
H, stats, st = P.solve(waves, rtol=1e-8, check_every=4)
print("ITERS", stats[0]["iters"], "STATUS", st, flush=True)
P.close()
ctx.close()
"""


def _run(level):
    env = dict(os.environ)
    env.pop("FEMH_LOG", None)
    if level is not None:
        env["FEMH_LOG"] = str(level)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], capture_output=True, text=True, env=env,
                       timeout=240)
    assert r.returncode == 0, r.stderr
    iters = int(re.search(r"ITERS (\d+)", r.stdout).group(1))
    return iters, [l for l in r.stderr.splitlines() if l.startswith("[femh]")]


def test_log_lines_follow_the_solve():
    iters, lines = _run(2)
    text = "\n".join(lines)
    assert re.search(r"problem 5x5x5: 216 active nodes, 648 unknowns", text), text
    assert re.search(r"solve: 648 unknowns, FP64, rtol 1\.0e-08", text), text
    chunk = [int(m.group(1)) for m in re.finditer(r"solve:   iteration (\d+), recursive", text)]
    assert chunk and chunk == sorted(chunk) and chunk[-1] == iters, (chunk, iters)
    assert re.search(r"segment stopped at iteration %d \(converged\)" % iters, text), text
    assert re.search(r"true \|b - Ax\|/\|b\| = [0-9.e+-]+ after %d iterations" % iters, text), text
    assert re.search(r"finished with status 0 after %d iterations" % iters, text), text


def test_nothing_is_logged_by_default():
    _, lines = _run(None)
    assert lines == []
