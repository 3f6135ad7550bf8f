"""Two tile schedules, one result: the FP32 MatVec with the J range split 1,
3 and 64 ways (the library's split-count override, read when it loads, so
each schedule runs in a child process) against the automatic split.  The
partial sums are grouped differently, so the results agree to FP32
rounding, not bit for bit; an indexing or synchronisation mistake in the
split handling would show as a large difference."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2503_02259_amd import workloads as W
from helpers import as_prec, colrel, oracle_rows

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CASES = [(20011, 3, 33), (5003, 3, 17), (3001, 8, 64)]

CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, ROOT)
import paper_2503_02259_amd as hg
from paper_2503_02259_amd import workloads as W
out = {}
for n, d, k in CASES:
    p = W.random_problem(n, d, 40 + k, l=0.2, f=1.1, s=0.02, k=k)
    X = torch.from_numpy(p.X.astype(np.float32)).cuda()
    V = torch.from_numpy(p.extra["V"].astype(np.float32)).cuda()
    out["%d_%d_%d" % (n, d, k)] = hg.kmatvec(X, V, 0, 0.2, 1.1, 0.02).cpu().numpy()
np.savez(sys.argv[1], **out)
"""


def _run(splits, path):
    env = dict(os.environ)
    env.pop("HIGP_F32_SPLITS", None)
    if splits:
        env["HIGP_F32_SPLITS"] = str(splits)
    code = CHILD.replace("ROOT", repr(ROOT)).replace("CASES", repr(CASES))
    print("schedule: %s J splits" % (splits or "automatic"), flush=True)
    subprocess.run([sys.executable, "-c", code, str(path)], env=env, check=True, timeout=300)
    return np.load(path)


def test_fp32_matvec_split_schedules_agree(tmp_path):
    auto = _run(0, tmp_path / "auto.npz")
    for splits in (1, 3, 64):
        got = _run(splits, tmp_path / ("s%d.npz" % splits))
        for key in auto.files:
            err = colrel(got[key], auto[key]).max()
            assert err <= 2e-6, (splits, key, err)
    for n, d, k in CASES:
        p = W.random_problem(n, d, 40 + k, l=0.2, f=1.1, s=0.02, k=k)
        X, V = as_prec(p.X, torch.float32), as_prec(p.extra["V"], torch.float32)
        rows = slice(n - 77, n)
        ref = oracle_rows(X, V, 0, 0.2, 1.1, 0.02, rows)
        assert colrel(auto["%d_%d_%d" % (n, d, k)][rows], ref).max() <= 1e-5
