"""The oracle's pins catch plausible mistakes: each case below plants one
mistake in a copy of oracle/gerbil_oracle.c (a wrong complement, the larger
strand taken as canonical, least-significant-first packing, a dropped last
window, an exclusive threshold, the wrong KMC2 exception, a short minimizer
window, a swapped base code, lower-case t rejected, a histogram off by one,
a complement without reversal), builds it with gcc, and runs the pin tests
against it in a child process. Every mutant must make a pin fail. Nothing
here touches the GPU library."""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

from conftest import ROOT

SRC = os.path.join(ROOT, "oracle", "gerbil_oracle.c")

# (name, text in gerbil_oracle.c, replacement): every occurrence is replaced;
# each text occurs once, except the threshold test, which the pair count and
# the pair output both make
MUTANTS = [
    ("complement", "case 'C': return 'G';", "case 'C': return 'C';"),
    ("canonical_is_max", "if (memcmp(t, s, k) < 0) c = t;", "if (memcmp(t, s, k) > 0) c = t;"),
    ("packing_lsb_first", "for (uint32_t j = 0; j < k; j++) w[j / 32] = (w[j / 32] << 2) | code2(s[j]);",
     "for (uint32_t j = 0; j < k; j++) w[j / 32] |= code2(s[j]) << (2 * (j % 32));"),
    ("dropped_last_window", "for (uint64_t i = 0; i + k <= L; i++) {\n            if (!window_ok(R + i, k)) continue;\n"
                            "            (*n_valid)++;",
     "for (uint64_t i = 0; i + k < L; i++) {\n            if (!window_ok(R + i, k)) continue;\n"
     "            (*n_valid)++;"),
    ("threshold_exclusive", "j - i >= threshold", "j - i > threshold"),
    ("kmc2_exception", 'memcmp(c, "ACA", 3) == 0', 'memcmp(c, "AAC", 3) == 0'),
    ("minimizer_window", "for (uint32_t j = 0; j + m <= k; j++) {", "for (uint32_t j = 0; j + m < k; j++) {"),
    ("base_code", "case 'C': return 1;\n        case 'G': return 2;", "case 'C': return 2;\n        case 'G': return 1;"),
    ("lowercase_t", "|| c == 'g' || c == 't';", "|| c == 'g';"),
    ("histogram_off_by_one", "out->hist[j - i]++;", "out->hist[j - i - 1]++;"),
    ("complement_not_reversed", "t[n - 1 - j] = complement(s[j]);", "t[j] = complement(s[j]);"),
]


def _run_mutant(tmp, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == (2 if name == "threshold_exclusive" else 1), f"mutation {name}: unexpected matches"
    src = os.path.join(tmp, f"{name}.c")
    lib = os.path.join(tmp, f"lib{name}.so")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", src, "-o", lib], check=True)
    env = dict(os.environ, ORACLE_LIBRARY=lib, HYPOTHESIS_PROFILE="default")
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, p.returncode, p.stdout[-400:]


def test_the_unmutated_oracle_passes_its_pins():
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stdout[-2000:]


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        with cf.ThreadPoolExecutor(max_workers=4) as ex:
            res = list(ex.map(lambda m: _run_mutant(tmp, *m), MUTANTS))
    survived = [(name, out) for name, rc, out in res if rc == 0]
    assert not survived, f"mutants that pass every pin: {[n for n, _ in survived]}"
    # a failing run is a failed test, not a crash of the runner or a collection error
    for name, rc, out in res:
        assert rc == 1, (name, rc, out)
