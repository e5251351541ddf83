"""The oracle's pins again, against a build of the same sources under
AddressSanitizer and UndefinedBehaviorSanitizer (host code): an out-of-bounds
access, a use after free or an undefined operation anywhere on the paths the
pins exercise aborts the run."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# every oracle pin file; the slowest parametrisations are left to the plain run
FILES = ["test_oracle_plan_layer.py", "test_oracle_physics.py", "test_oracle_robot.py", "test_oracle_cem.py",
         "test_oracle_random.py", "test_oracle_mlp.py", "test_oracle_region.py", "test_oracle_dr.py",
         "test_oracle_early_stop.py", "test_oracle_movepush.py", "test_oracle_pickplace_box.py",
         "test_oracle_cull_and_counter.py"]
SKIP = "not training_fits and not face_cull and not (reduction_over_scenarios and max)"


def test_pins_pass_under_address_and_undefined_behaviour_sanitizers():
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("no gcc to build the sanitized oracle")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan is not installed")
    subprocess.run(["sh", os.path.join(ROOT, "oracle", "build.sh"), "sanitize"], check=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               CEM_ORACLE_LIB=os.path.join(ROOT, "oracle", "liboracle_san.so"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "-k", SKIP] + [os.path.join(ROOT, "tests", f) for f in FILES],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "passed" in r.stdout
