"""The CPU oracle's C code under AddressSanitizer and
UndefinedBehaviorSanitizer: ``sanitize_oracle.c`` drives every oracle entry
point (count, shards, query keys, traversal, merge, pruning, localisation)
on random reads with N, lowercase, empty and short reads at k = 1..127;
any out-of-bounds access, leak or undefined operation aborts it.  Skipped
where the compiler has no sanitizer runtime."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE = os.path.join(ROOT, "oracle")
SRCS = [os.path.join(ORACLE, f) for f in
        ("oracle.c", "traverse.c", "merge.c", "prune.c", "localize.c")]
FLAGS = ["-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]


def _sanitizer_available(tmp_path) -> bool:
    if shutil.which("gcc") is None:
        return False
    src = tmp_path / "probe.c"
    src.write_text("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", str(src), "-o",
                        str(tmp_path / "probe")], capture_output=True)
    return r.returncode == 0 and subprocess.run([str(tmp_path / "probe")]).returncode == 0


def test_oracle_under_sanitizers(tmp_path):
    if not _sanitizer_available(tmp_path):
        pytest.skip("gcc has no AddressSanitizer/UBSan runtime here")
    exe = tmp_path / "sanitize_oracle"
    subprocess.check_call(["gcc"] + FLAGS + ["-o", str(exe),
                                             os.path.join(HERE, "sanitize_oracle.c")]
                          + SRCS)
    env = dict(os.environ, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle run ok" in r.stdout
    assert "runtime error" not in r.stderr
