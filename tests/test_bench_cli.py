"""The benchmark's command line without a GPU, and the algorithmic flop
counts its roofline uses (hand-counted from the two tableaux)."""
import json
import os
import subprocess
import sys

import pytest

from paper_2210_12375_amd import roofline as rl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        *args], capture_output=True, text=True, timeout=300,
                       cwd=ROOT)
    return r.returncode, r.stdout.strip().splitlines()


def test_more_than_one_gpu_is_refused():
    rc, out = run_bench("--gpus", "2")
    assert rc == 2
    assert "one GPU" in json.loads(out[-1])["error"]


def test_no_gpu_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    rc, out = run_bench("--steps", "1", "--warmup", "0")
    assert rc == 3
    assert "error" in json.loads(out[-1])


@pytest.mark.parametrize("method,flops", [
    # Dormand-Prince: 20 nonzero a_sj (s = 2..7; b_2 = 0), 6 nonzero
    # error weights (e_2 = 0); Van der Pol f = 5 flops, n = 2:
    # 2 (2*20 + 12) + 6*5 + 2 (2*6 + 1) + (6*2 + 2) + 6 = 180
    ("dopri5", 180),
    # Tsitouras: 21 nonzero a_sj (b_7 = 0 is not a stage input), 7 error
    # weights: 2 (2*21 + 12) + 30 + 2 (2*7 + 1) + 14 + 6 = 188
    ("tsit5", 188),
])
def test_flops_per_attempt_hand_count(method, flops):
    assert rl.flops_per_attempt(method, 2, rl.VDP_FLOPS) == flops
