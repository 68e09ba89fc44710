"""The FP64 oracle's C++ library under AddressSanitizer, on the calls the
benchmark makes: each ensemble member's accuracy check (256 points, the
oracle's OpenMP threads) and the CPU baseline's single-threaded pieces of at
most 256 points, plus the composite loss of the Burgers training set.  The
library is rebuilt with -fsanitize=address into a scratch directory and
loaded by a child interpreter with the sanitizer runtime preloaded; a heap
overrun, use after free or double free fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r'''
import sys
sys.path.insert(0, sys.argv[1])
sys.path.insert(1, sys.argv[2])
import numpy as np
import oracle
assert oracle._LIB_PATH.startswith(sys.argv[1]), oracle._LIB_PATH
import pinn_inputs as pi
ch = pi.CHANNELS["burgers"]
ens = pi.make_ensemble(seed=0)
for m in ens:
    ref = oracle.evaluate(m.params, m.x[:256], ch, "burgers", (m.nu,), want_jets=False)
    assert np.isfinite(ref.grad).all()
for m in ens[::8]:
    n = max(1, int(np.ceil(0.002 * m.N)))
    for a in range(0, n, 256):
        oracle.evaluate(m.params, m.x[a:min(n, a + 256)], ch, "burgers", (m.nu,), want_jets=False, threads=1)
ts = pi.burgers_training_set(seed=0)
oracle.evaluate_segments(ts.params, ts.x, ch, "burgers", ts.coef, ts.segments)
print("oracle calls clean")
'''


@pytest.mark.skipif(not shutil.which("g++") or not shutil.which("gcc"), reason="needs g++")
def test_oracle_under_address_sanitizer(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime")
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "oracle", "__init__.py"), pkg / "__init__.py")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-fsanitize=address", "-fno-omit-frame-pointer", "-o", str(pkg / "liborc.so"),
                    os.path.join(ROOT, "oracle", "pinn_oracle.cpp")], check=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", CHILD, str(tmp_path), ROOT], capture_output=True, text=True,
                       env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out, out[-4000:]
    assert "oracle calls clean" in out, out[-2000:]
