"""The oracle built with AddressSanitizer + UndefinedBehaviorSanitizer
(oracle/run_sanitized_tests.sh runs the whole CPU suite that way): a
subprocess with the sanitizer runtimes preloaded runs the fit (both update
rules), the adjoint and the loss gradient on small inputs and must end
cleanly with the same bits as the ordinary build."""
import hashlib
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import hashlib, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import gs_oracle
rng = np.random.default_rng(5)
c = rng.uniform(0, 40, size=(6, 3))
x = c[rng.integers(0, 6, 3000)] + 2.5 * rng.standard_normal((3000, 3))
h = hashlib.sha256()
for rule in ("parallel", "sequential"):
    r = gs_oracle.fit(x, 3.0, 100, rule=rule)
    for a in (r.labels, r.counts, r.sums, r.keys, r.m_hist):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(repr((r.K, r.n_iter, r.flags)).encode())
L, g, _, _ = gs_oracle.loss_and_grad(x[:400], 2.0, 50)
h.update(np.float64(L).tobytes())
h.update(np.ascontiguousarray(g).tobytes())
print(h.hexdigest())
"""


def _run(env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    res = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    return res.stdout.strip().splitlines()[-1]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_sanitized_oracle_runs_clean_and_matches():
    from oracle import gs_oracle

    gs_oracle.build(sanitize=True)
    gs_oracle.build(sanitize=False)
    rt = [subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
          for n in ("libasan.so", "libubsan.so")]
    if not all(os.path.isabs(p) and os.path.exists(p) for p in rt):
        pytest.skip("sanitizer runtimes not installed")
    plain = _run({"GS_ORACLE_SANITIZE": "0"})
    san = _run({"GS_ORACLE_SANITIZE": "1", "LD_PRELOAD": " ".join(rt),
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    assert san == plain
