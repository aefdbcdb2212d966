"""Runs the oracle's CPU pins against its AddressSanitizer +
UndefinedBehaviorSanitizer build (host code only, on the CPU).

    python oracle/sanitize_check.py [pytest args]

Builds ``oracle/liboracle_san.so``, then starts pytest on the pin files in a
child process with the ASan runtime preloaded (a sanitized shared library
loaded into an unsanitized Python needs its runtime first) and
NAUTICLE_ORACLE_LIB pointing at the sanitized build.  Any sanitizer report
aborts the child; the exit status is pytest's.  Leak detection is off (the
interpreter itself is not leak-clean)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_pins_ex1a.py", "tests/test_oracle_pins_laws.py",
        "tests/test_oracle_pins_ch.py", "tests/test_oracle_pins_verlet.py"]


def main(argv):
    sys.path.insert(0, ROOT)
    from oracle import build

    lib = build.build(sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], check=True, capture_output=True,
                          text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], check=True, capture_output=True,
                           text=True).stdout.strip()
    env = dict(os.environ)
    env["LD_PRELOAD"] = " ".join([asan, ubsan])
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["NAUTICLE_ORACLE_LIB"] = lib
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider"] + PINS + list(argv)
    return subprocess.run(cmd, cwd=ROOT, env=env).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
