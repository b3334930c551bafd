"""The C oracle and the C read generator under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/sanitize_driver.c runs their entry points
on small seeded inputs (every k class from 1 to 479 words, both strands
modes, shards, the key lookups, the encoder, both minimizer orders, the
record codec). Host code only, built with gcc."""
import os
import shutil
import subprocess
import tempfile

import pytest

from conftest import ROOT


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_and_generator_are_clean_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "sanitized")
        subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "sanitize_driver.c"),
                        os.path.join(ROOT, "oracle", "gerbil_oracle.c"), os.path.join(ROOT, "synth", "synth.c"),
                        "-o", exe, "-lm", "-lpthread"], check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
        p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
        assert "ok" in p.stdout
