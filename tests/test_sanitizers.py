"""CPU: the oracle and the library's host runtime built with AddressSanitizer and
UndefinedBehaviorSanitizer, each run in a child process with its sanitizer runtime
preloaded over the CPU tests that exercise it.  For the library that is its host code
(argument checks, tile planning, the field files, host-side draws and orientations);
no kernel runs and no GPU is needed.  A sanitizer report or a failing test fails here."""
import os
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))

REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer", "SUMMARY: UndefinedBehaviorSanitizer")


def _pytest(env_extra, args, logdir, timeout=1200):
    """pytest over `args` in a child process; the sanitizers write their reports to files
    under logdir (the child's own output capture would lose a report written as it exits)."""
    env = dict(os.environ, **env_extra)
    env.pop("PYTEST_ADDOPTS", None)
    log = str(Path(logdir) / "sanitizer")
    env["ASAN_OPTIONS"] = f"detect_leaks=0:abort_on_error=1:log_path={log}"
    env["UBSAN_OPTIONS"] = f"halt_on_error=1:print_stacktrace=1:log_path={log}"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *args],
                       cwd=str(ROOT), env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    for f in sorted(Path(logdir).glob("sanitizer*")):
        out += f"\n--- {f.name}\n" + f.read_text(errors="replace")
    return r.returncode, out


def _clean(rc, out):
    assert rc == 0, out[-4000:]
    bad = [m for m in REPORTS if m in out]
    assert not bad, out[-4000:]
    assert " passed" in out, out[-2000:]


def test_oracle_under_asan_and_ubsan(tmp_path):
    import oracle
    lib = oracle.build(force=True, sanitize=True, out=tmp_path / "liboracle_san.so")
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    # every pin except the long relaxations (each routine they call is covered by the rest)
    keep = ("not power_rule_trace and not gradient_flow_descends and not fall_at_fourth_order "
            "and not converges_at_fourth_order and not shadow_energy")
    rc, out = _pytest({"SKYR_ORACLE_LIB": str(lib), "LD_PRELOAD": asan, "OMP_NUM_THREADS": "4"},
                      ["tests/test_oracle_pins.py", "-k", keep], tmp_path)
    _clean(rc, out)


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    from paper_2604_25876_amd import build
    lib = build.build_sanitized(tmp_path / "libskyr_san.so")
    # the default-tile restatement follows the full shape list, which this build leaves out
    rc, out = _pytest({"SKYR_LIB": str(lib), "LD_PRELOAD": build.asan_runtime()},
                      ["tests/test_abi.py", "tests/test_files.py", "-k", "not default_tile"], tmp_path)
    _clean(rc, out)
