"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU): the
library's host C++ built with both sanitizers (every finding fatal) runs the
CPU tests of the C-ABI (exports, reference matrices, clustering against the
oracle, configuration errors, the host Godunov flux and its reverse mode) in
a child process with the ASan runtime preloaded; the reference-matrix
generator, built the same way, must write the header of the regular build
byte for byte."""
import os
import subprocess
import sys
import tempfile

import pytest

from paper_2202_10313_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FINDINGS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


@pytest.fixture(scope="module")
def sanitized():
    try:
        return build.build_sanitized_host()
    except RuntimeError as e:   # no g++ sanitizer runtime in this environment
        pytest.skip(f"sanitized build unavailable: {e}")


def _clean(text):
    return not any(f in text for f in FINDINGS)


def test_generator_under_sanitizers_writes_the_same_header(sanitized):
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "refmats.h")
        r = subprocess.run([sanitized["gen"], out, "2", "3", "4", "5"], capture_output=True, text=True)
        assert r.returncode == 0 and _clean(r.stdout + r.stderr), r.stderr[-4000:]
        with open(out, "rb") as f, open(os.path.join(build.CSRC, "generated", "refmats.h"), "rb") as g:
            assert f.read() == g.read()


def test_host_library_tests_under_sanitizers(sanitized):
    env = dict(os.environ, EDG_LIBRARY=sanitized["lib"], LD_PRELOAD=sanitized["runtime"],
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    # the child loads the instrumented library, not the regular one
    probe = ("from paper_2202_10313_amd import binding; binding.lib(); "
             "print([l.split()[-1] for l in open('/proc/self/maps') if 'libedge_lts' in l][0])")
    r = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, env=env, cwd=ROOT, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == sanitized["lib"], r.stdout + r.stderr[-2000:]
    files = [os.path.join(ROOT, "tests", f) for f in ("test_host_library.py", "test_host_flux.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + files,
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    text = r.stdout + r.stderr
    print(text[-1500:])
    assert r.returncode == 0 and _clean(text), text[-4000:]
    assert " passed" in r.stdout
