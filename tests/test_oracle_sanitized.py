"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc) runs every CPU pin of the solver and segmentation oracles without a
finding: no out-of-bounds access, use after free or undefined behaviour in the
code the GPU path is judged against."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_pins_pass_under_address_and_ub_sanitizers(tmp_path):
    from oracle import build
    try:
        lib = build.build(sanitize=True, out=str(tmp_path / "liboracle_asan.so"))
        runtime = build.asan_runtime()
    except (OSError, subprocess.CalledProcessError) as e:
        pytest.skip(f"no sanitizer toolchain: {e}")
    if not os.path.isabs(runtime) or not os.path.exists(runtime):
        pytest.skip("gcc has no AddressSanitizer runtime")
    report = tmp_path / "asan"
    env = dict(os.environ, LD_PRELOAD=runtime, ABC_ORACLE_LIB=lib,
               ASAN_OPTIONS=f"detect_leaks=0:abort_on_error=1:log_path={report}",
               UBSAN_OPTIONS=f"print_stacktrace=1:log_path={report}")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"), os.path.join(ROOT, "tests", "test_oracle_seg.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    found = sorted(p.name for p in tmp_path.iterdir() if p.name.startswith("asan"))
    reports = "".join((tmp_path / f).read_text()[:2000] for f in found)
    assert r.returncode == 0 and not found, f"{r.stdout[-2000:]}\n{r.stderr[-2000:]}\n{reports}"
    assert " passed" in r.stdout
