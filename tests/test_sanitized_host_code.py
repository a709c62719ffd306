"""The host C code (the oracle and the input generators) built with
AddressSanitizer and UndefinedBehaviorSanitizer, then driven by their own
tests in a child process that preloads the sanitizer runtimes (no GPU)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ("-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g")

RUNNER = r"""
import subprocess, sys
sys.path.insert(0, {root!r})
import inputs, oracle
oracle._lib = oracle.load(oracle.build(force=True, out={orc!r}, extra={san!r}))
subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", *{san!r},
                       {gen_src!r}, "-o", {gen!r}, "-lm"])
inputs._LIB = {gen!r}
inputs._lib = None
import pytest
sys.exit(pytest.main([{pins!r}, {inp!r}, "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"]))
"""


def runtime(name):
    path = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_and_generators_under_sanitizers(tmp_path):
    asan, ubsan = runtime("libasan.so"), runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    code = RUNNER.format(root=ROOT, orc=str(tmp_path / "liboracle_san.so"), san=SAN,
                         gen_src=os.path.join(ROOT, "inputs", "gen.c"), gen=str(tmp_path / "libspkgen_san.so"),
                         pins=os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                         inp=os.path.join(ROOT, "tests", "test_inputs.py"))
    env = dict(os.environ, LD_PRELOAD=asan + " " + ubsan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), env=env, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
