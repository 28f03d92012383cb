"""The oracle and the input generator under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is the ground truth of every parity test, so its C code (and the generator's) is run
instrumented: a child process builds both libraries with -fsanitize=address,undefined
(DBL_SANITIZE=1 selects those builds), preloads the ASan runtime into the Python interpreter
and runs the oracle's pins (the paper's worked examples, brute force on small graph families,
the large-graph view) and the generator tests. Any out-of-bounds access, use after free or
undefined behaviour aborts the child and fails this test. Leak checking is off: the
interpreter itself keeps memory until exit.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    gcc = shutil.which("gcc")
    if not gcc:
        return None
    p = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_and_generator_pins_under_asan_ubsan(tmp_path):
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    env = dict(os.environ)
    env.update(DBL_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               DBLGEN_CACHE=str(tmp_path / "cache"), PYTHONDONTWRITEBYTECODE="1")
    # build the instrumented libraries first (without the preload, so gcc is not instrumented)
    build_env = dict(env)
    build_env.pop("LD_PRELOAD")
    subprocess.run([sys.executable, "-c", "import oracle, dblgen; oracle.build(); dblgen.build()"],
                   cwd=ROOT, env=build_env, check=True)
    # the child really runs the instrumented libraries with the ASan runtime mapped
    probe = ("import oracle, dblgen, numpy as np\n"
             "o = oracle.OracleIndex(3, [0, 1], [1, 2]).build(k=1, kp=2)\n"
             "assert o.query_truth([0], [2])[0] == 1\n"
             "dblgen.make_rmat_workload('probe', 6, 1, draws=256, n_insert=4, n_query=4)\n"
             "maps = open('/proc/self/maps').read()\n"
             "assert 'liboracle_san.so' in maps and 'libdblgen_san.so' in maps, 'not instrumented'\n"
             "assert 'libasan' in maps and 'libubsan' in maps, 'no sanitizer runtime'\n")
    subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, check=True)
    tests = ["tests/test_oracle_paper.py", "tests/test_oracle_brute.py",
             "tests/test_oracle_scale.py", "tests/test_oracle_big.py", "tests/test_gen.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *tests], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1500)
    tail = (r.stdout[-3000:] + "\n" + r.stderr[-3000:])
    assert r.returncode == 0, f"sanitized run failed:\n{tail}"
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr, tail
    assert "runtime error" not in r.stderr, tail
