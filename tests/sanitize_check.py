"""Host AddressSanitizer + UndefinedBehaviorSanitizer run of the CPU suite.

Builds the library's host code (hipcc -Xarch_host -fsanitize=...) and the
CPU oracle (clang++ -fsanitize=address,undefined) with the sanitizers, runs
`pytest -m "not gpu"` against them with the sanitizer runtime preloaded
(leak detection off: the interpreter itself holds its allocations), then
rebuilds both normally.  CPU only: nothing here runs device code.

    python tests/sanitize_check.py
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main() -> int:
    import oracle
    from paper_1801_09847_amd import _build
    try:
        _build.build(verbose=True, sanitize=True)
        oracle.build(force=True, sanitize=True)
        env = dict(os.environ, LD_PRELOAD=_build.ASAN_RUNTIME,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:strict_string_checks=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        return subprocess.call([sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                                os.path.join(ROOT, "tests")], env=env, cwd=ROOT)
    finally:
        _build.build()
        oracle.build(force=True)


if __name__ == "__main__":
    sys.exit(main())
