"""Host-side checks of bench.py: the argument sets the benchmark is run with,
the one-GPU guard and the algorithmic byte model (no GPU needed)."""
import subprocess
import sys

import pytest

import bench


def test_driver_argument_set_parses():
    a = bench.parse_args(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (a.gpus, a.steps, a.warmup, a.config) == (1, 20, 5, "large")
    a = bench.parse_args([])
    assert a.steps >= 1 and a.warmup >= 0 and a.config == "large"
    a = bench.parse_args(["--steps", "3", "--warmup", "0", "--config", "production", "--no-batch",
                          "--no-adjoint", "--no-cpu-baseline", "--no-production"])
    assert a.config == "production" and a.no_batch and a.no_production


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", str(n)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stage_bytes_sum_to_the_step_model():
    # the step's algorithmic bytes at 256^3/768^3 (the per-stage model):
    # deposit 16 Np + R, r2c R + C, y 2C, Green 3C, inverse y 2C + 3C,
    # c2r 3(C + R), kick/drift 72 Np + 12 min(M, 8 Np), sort 32 Np
    sb = bench.stage_bytes(256, 768)
    n_p, M = 256 ** 3, 768 ** 3
    R, C = 4 * M, 8 * 768 * 768 * 385
    want = 16 * n_p + R + (R + C) + 2 * C + 3 * C + 2 * C + 3 * C + 3 * (C + R) \
        + 72 * n_p + 12 * min(M, 8 * n_p) + 32 * n_p
    assert sum(sb.values()) == want


def test_cycled_schedule_counts_steps():
    calls = []

    class FakeSim:
        def init_2lpt(self, seed, k, p):
            calls.append(("init",))

        def step(self, a0, a1):
            calls.append(("step", a0, a1))

    class Cfg:
        nstep, seed = 10, 1

    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("host-only check")
    orig = torch.cuda.synchronize
    torch.cuda.synchronize = lambda *a, **k: None
    try:
        e = list(range(11))
        bench.cycled_steps(FakeSim(), Cfg, (None, None), e, 23)
    finally:
        torch.cuda.synchronize = orig
    assert sum(1 for c in calls if c[0] == "step") == 23
    assert sum(1 for c in calls if c[0] == "init") == 3
    # every pass restarts at the first step of the schedule
    firsts = [calls[i + 1] for i, c in enumerate(calls) if c[0] == "init"]
    assert all(f == ("step", 0, 1) for f in firsts)
