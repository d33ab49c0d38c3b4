"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) runs its pins and a workload sample cleanly, with results
identical to the ordinary build."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2208_09985_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(_asan_runtime() is None, reason="gcc has no AddressSanitizer runtime here")
def test_oracle_pins_and_sample_under_sanitizers(tmp_path):
    san = oracle.build(sanitize=True)
    env = dict(os.environ, SCG_ORACLE_LIB=san, LD_PRELOAD=_asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the pins themselves, against the sanitized build
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    # a workload sample, compared with the ordinary build
    out = tmp_path / "san.npz"
    code = ("import numpy as np, oracle; from paper_2208_09985_amd import synth; "
            "b = synth.make_batch('uneven_lognormal', 24); r = oracle.align_batch(b, 64, 24, 64, threads=4); "
            f"np.savez({str(out)!r}, edits=r['edits'], text_end=r['text_end'], ops=r['ops'], n_ops=r['n_ops'])")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    got = np.load(out)
    ref = oracle.align_batch(synth.make_batch("uneven_lognormal", 24), 64, 24, 64, threads=4)
    for key in ("edits", "text_end", "ops", "n_ops"):
        assert np.array_equal(got[key], ref[key]), key
