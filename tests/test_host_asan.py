"""The library's host code under AddressSanitizer, on a machine without a GPU.

Every library source is compiled for the host only (no device code) with
AddressSanitizer and linked against a stand-in HIP runtime
(tests/host_asan/fake_hip.cpp) that checks each kernel launch's configuration,
each grouped launch's member table and every device pointer it is handed,
while the kernels themselves do not run.  The driver (tests/host_asan/driver.cpp)
walks the ensemble step exactly as the benchmark drives it, under several
synthetic clocks so that the autotuners take different choices, then single
plans of every PDE kind, operand type and tuning, composite losses, the
modified MLP, graphs, the tuning cache and the no-allocation step.  A heap
overrun, use after free, leak, invalid launch or leftover stream, event, graph
or allocation fails the test."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

import pinn_inputs as pi

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "paper_2606_29702_amd", "csrc")
HARNESS = os.path.join(HERE, "host_asan")
OUT = os.path.join(HARNESS, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
# host-only compilation; the sanitizer applies to the host pass only
FLAGS = ["-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
         "-Xarch_host", "-fsanitize=address", "-fno-omit-frame-pointer",
         "-I", os.path.join(ROOT, "include"), "-I", SRC]


def _newest_source():
    return max(os.path.getmtime(os.path.join(d, f)) for d in (SRC, HARNESS, os.path.join(ROOT, "include"))
               for f in os.listdir(d) if f.endswith((".hip", ".cpp", ".hpp", ".h")))


def _compile(src, newest):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    if os.path.exists(obj) and os.path.getmtime(obj) >= newest:
        return obj
    r = subprocess.run([HIPCC] + FLAGS + ["-c", src, "-o", obj], capture_output=True, text=True)
    assert r.returncode == 0, f"host compile of {src} failed:\n{r.stderr[-3000:]}"
    return obj


def _build():
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(os.path.join(SRC, f) for f in os.listdir(SRC) if f.endswith((".hip", ".cpp")))
    srcs += [os.path.join(HARNESS, "fake_hip.cpp"), os.path.join(HARNESS, "driver.cpp")]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, _newest_source()), srcs))
    # host-only objects name their (absent) device images; empty stand-ins
    names = set()
    for o in objs:
        r = subprocess.run(["nm", "-u", o], capture_output=True, text=True, check=True)
        names.update(w for w in r.stdout.split() if w.startswith("__hip_fatbin"))
    stub_c = os.path.join(OUT, "fatbin_stubs.c")
    with open(stub_c, "w") as f:
        f.writelines(f"char {n}[64];\n" for n in sorted(names))
    stub_o = os.path.join(OUT, "fatbin_stubs.o")
    subprocess.run(["gcc", "-c", stub_c, "-o", stub_o], check=True)
    exe = os.path.join(OUT, "driver")
    r = subprocess.run([CLANG, "-fsanitize=address", "-o", exe] + objs + [stub_o, "-lpthread"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG) and shutil.which("nm")),
                    reason="needs hipcc, clang++ and nm")
def test_host_paths_under_address_sanitizer(tmp_path):
    exe = _build()
    shapes = tmp_path / "ensemble_shapes.txt"
    with open(shapes, "w") as f:
        for m in pi.make_ensemble(seed=0, with_points=False):
            dims = [2] + [m.width] * m.hidden + [1]
            f.write(f"{m.N} {m.nu!r} " + " ".join(map(str, dims)) + "\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1")
    r = subprocess.run([exe, str(shapes), str(tmp_path / "tuning_cache.txt")], capture_output=True, text=True,
                       env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert "host paths OK" in out, out[-2000:]
