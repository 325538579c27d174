"""Launch-geometry check of every main call sequence on the CPU (BM_DRY_RUN=1):
each kernel launch is compared with the allocations it would touch."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def test_dry_run_call_sequences():
    env = dict(os.environ, BM_DRY_RUN="1")
    r = subprocess.run([sys.executable, os.path.join(HERE, "dry_run_flow.py")], env=env,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "dry run ok" in r.stdout
