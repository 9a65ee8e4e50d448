"""bench.py's command line on the CPU: it measures one GPU only and says so
for any other count, before touching a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_switches():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--no-cpu-baseline", "--no-serve"):
        assert flag in r.stdout


def test_matrix_core_flops_follow_each_path_operands():
    # Per step, in units of 2*B*H*N*d^2.  bf16 applies S as hi + lo in the
    # apply (2); the fused query backward takes X = S G as hi + lo below
    # d = 128 and as the hi part at d = 128, plus the dS product; fp32
    # applies S as one operand everywhere.
    sys.path.insert(0, ROOT)
    import bench
    one = {"launches_per_step": 1.0}
    bf16_step = {k: one for k in ("summary_fwd", "apply", "bwd_query_ds", "bwd_key")}
    fp32_step = {k: one for k in ("summary_fwd", "apply", "bwd_query", "summary_bwd", "bwd_key")}
    unit = lambda d: 2 * d  # elems = 1
    assert bench.mma_flops_per_step(bf16_step, "bf16", 1, 128) == 7 * unit(128)
    assert bench.mma_flops_per_step(bf16_step, "bf16", 1, 64) == 8 * unit(64)
    assert bench.mma_flops_per_step(fp32_step, "fp32", 1, 128) == 6 * unit(128)
    # combine and the image builder do no products of the method
    assert bench.mma_flops_per_step({"combine": {"launches_per_step": 2.0}}, "bf16", 1, 128) == 0
