"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (gcc, CPU
only): a driver (oracle_sanitize_driver.c) runs oracle_ccg and oracle_residual through
the stop test, a restart, the rank step and the traces, in both the FP64 and the
extended build; any out-of-bounds access, leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "oracle", "ccg_oracle.c")
DRIVER = os.path.join(HERE, "oracle_sanitize_driver.c")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
@pytest.mark.parametrize("real", ["double", "long double"])
def test_oracle_is_clean_under_asan_ubsan(tmp_path, real):
    exe = str(tmp_path / "orc_san")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           f"-DORC_REAL={real}", "-o", exe, SRC, DRIVER, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    lines = [l for l in r.stdout.splitlines() if l.startswith("n=")]
    assert len(lines) == 6
    assert any("restarts=0" not in l for l in lines)        # a restart ran
    assert any("deflations=0" not in l for l in lines)      # the rank step dropped agents
    assert any("reinflations=0" not in l for l in lines)    # and agents were re-inflated
