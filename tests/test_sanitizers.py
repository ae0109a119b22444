"""Host code under the host compiler's address and undefined-behaviour
sanitizers (no GPU): the library's argument checks (plain C++, the same source
the library links) against random and malformed batches, and the CPU oracle and
the input generators on ligands of 1 to 64 atoms.  Any out-of-bounds access,
use after free, leak or undefined behaviour aborts the test program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all", "-D_GLIBCXX_SANITIZE_VECTOR"]


def build_and_run(tmp_path, name, sources, extra=()):
    exe = str(tmp_path / name)
    cmd = ["g++", *SAN, *extra, *[os.path.join(ROOT, s) for s in sources], "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # the environment is passed on unchanged; ASan is told not to insist on being
    # first in the initial library list
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_checks_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "host_checks_fuzz",
                        ["paper_2303_06150_amd/csrc/host_checks.cpp", "tests/native/host_checks_fuzz.cpp"],
                        ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2303_06150_amd", "csrc")])
    assert "no sanitizer findings" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_and_generators_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "oracle_fuzz", ["oracle/oracle.cpp", "gen/gen.cpp", "tests/native/oracle_fuzz.cpp"],
                        ["-ffp-contract=off", "-mfma"])
    assert "no sanitizer findings" in out
