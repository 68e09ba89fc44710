"""C-ABI checks that need no GPU: the library loads, exports every function
the public header declares, and rejects bad arguments on the host before any
device work (status codes and messages)."""
import ctypes
import os
import re

import pytest

from paper_2606_29702_amd import _lib
from paper_2606_29702_amd._lib import Net, Pde, lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pinn_jet.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pinn_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported():
    names = declared_functions()
    assert len(names) >= 9
    so = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(so, n), n
    assert sorted(_lib.EXPORTS) == names


def _net(dims, ptr=1):
    d = (ctypes.c_int32 * len(dims))(*dims)
    L = len(dims) - 1
    W = (ctypes.c_void_p * L)(*([ptr] * L))
    b = (ctypes.c_void_p * L)(*([ptr] * L))
    n = Net(L, ctypes.cast(d, ctypes.POINTER(ctypes.c_int32)),
            ctypes.cast(W, ctypes.POINTER(ctypes.c_void_p)), ctypes.cast(b, ctypes.POINTER(ctypes.c_void_p)))
    return n, (d, W, b)


def _pde(kind, *coef):
    p = Pde()
    p.kind = kind
    for i, c in enumerate(coef):
        p.coef[i] = c
    return p


def create(dims, kind=1, coef=(0.003,), max_points=1024, prec=0, flags=0, cap=0, out=True):
    net, keep = _net(dims)
    h = ctypes.c_void_p()
    st = lib.pinn_plan_create(ctypes.byref(net), ctypes.byref(_pde(kind, *coef)), max_points, prec, flags,
                              cap, ctypes.byref(h) if out else None)
    return st, lib.pinn_last_error().decode()


@pytest.mark.parametrize("dims,kind,coef,kw,status,msg", [
    ([2, 32, 32, 1], 9, (1.0,), {}, -1, "unknown PDE kind"),
    ([3, 32, 32, 1], 1, (0.01,), {}, -1, "dims[0]"),
    ([2, 32, 32, 2], 1, (0.01,), {}, -1, "outputs"),
    ([2, 32, 32, 1], 2, (100.0,), {}, -1, "outputs"),
    ([2, 48, 48, 1], 1, (0.01,), {}, -2, "multiple of 32"),
    ([2, 32, 64, 1], 1, (0.01,), {}, -2, "equal"),
    ([2, 1024, 1], 1, (0.01,), {}, -2, "multiple of 32"),
    ([2, 1], 1, (0.01,), {}, -1, "n_layers"),
    ([2, 32, 32, 1], 1, (0.01,), {"max_points": 0}, -1, "max_points"),
    ([2, 32, 32, 1], 1, (0.01,), {"prec": 7}, -1, "precision"),
    ([2, 32, 32, 1], 1, (0.01,), {"flags": 8}, -1, "flags"),
    ([2, 32, 32, 1], 1, (float("nan"),), {}, -1, "finite"),
    ([2, 128, 128, 3], 2, (0.0,), {}, -1, "Reynolds"),
    ([2, 32, 32, 1], 1, (0.01,), {"out": False}, -1, "out is NULL"),
    ([2, 32, 32, 32, 1], 1, (0.01,), {"cap": 1000}, -6, "save_cap_bytes"),
])
def test_plan_create_rejects(dims, kind, coef, kw, status, msg):
    st, err = create(dims, kind, coef, **kw)
    assert st == status, (st, err)
    assert msg in err


def test_null_arguments():
    assert lib.pinn_plan_destroy(None) == -1
    assert lib.pinn_jet_forward(None, None, None, 1, None, None) == -1
    assert "plan is NULL" in lib.pinn_last_error().decode()
    assert lib.pinn_plan_create(None, None, 1, 0, 0, 0, None) == -1
    assert lib.pinn_jet_residual(None, None, None, None, 1, None, None, None, None, None) == -1
    assert lib.pinn_jet_backward(None, None, None, None, 1, None, None, None, None, None, None) == -1


def test_null_weight_pointer():
    net, keep = _net([2, 32, 32, 1], ptr=0)
    h = ctypes.c_void_p()
    st = lib.pinn_plan_create(ctypes.byref(net), ctypes.byref(_pde(1, 0.01)), 16, 0, 0, 0, ctypes.byref(h))
    assert st == -1 and "NULL" in lib.pinn_last_error().decode()


def test_channel_and_residual_counts():
    assert [lib.pinn_pde_channels(k) for k in (1, 2, 3, 4, 5, 6)] == [4, 5, 6, 8, 6, 1]
    assert [lib.pinn_pde_residuals(k) for k in (1, 2, 3, 4, 5, 6)] == [1, 3, 1, 1, 1, 1]
    assert lib.pinn_pde_channels(0) == 0


def test_oracle_and_library_share_no_code():
    """The oracle (test infrastructure) and the HIP library import or include
    nothing of each other."""
    pkg = os.path.join(ROOT, "paper_2606_29702_amd")
    orc = os.path.join(ROOT, "oracle")
    pat = re.compile(r"^\s*(#\s*include|import|from)\b.*$", re.M)
    for d, other in ((pkg, ("oracle", "pinn_oracle")), (orc, ("paper_2606_29702_amd", "pinn_jet", "jet_math",
                                                            "dev_common", "kernels.hpp"))):
        for dirpath, _, files in os.walk(d):
            for f in files:
                if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                    for line in pat.findall(open(os.path.join(dirpath, f)).read()):
                        for o in other:
                            assert o not in line, (f, line)


def test_single_hip_runtime_in_process():
    """The library binds to the HIP runtime torch loaded (one runtime per process)."""
    maps = set(l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l)
    assert len(maps) == 1, maps


def test_adam_step_rejects_bad_arguments():
    """Host-side validation of pinn_adam_step: nothing reaches the device."""
    from paper_2606_29702_amd._lib import Adam
    dims = (ctypes.c_int32 * 3)(2, 4, 1)
    hp = Adam(1e-3, 0.9, 0.999, 1e-8)
    assert lib.pinn_adam_step(2, dims, None, None, None, None, None, None, None, None, 1, ctypes.byref(hp),
                              None) == -1
    assert "NULL" in lib.pinn_last_error().decode()
    assert lib.pinn_adam_step(0, dims, None, None, None, None, None, None, None, None, 1, ctypes.byref(hp),
                              None) == -1
    one = (ctypes.c_void_p * 2)(ctypes.c_void_p(16), ctypes.c_void_p(16))
    pp = ctypes.cast(one, ctypes.POINTER(ctypes.c_void_p))
    assert lib.pinn_adam_step(2, dims, pp, pp, pp, pp, pp, pp, pp, pp, 0, ctypes.byref(hp), None) == -1
    assert "step" in lib.pinn_last_error().decode()
    bad = Adam(1e-3, 1.0, 0.999, 1e-8)
    assert lib.pinn_adam_step(2, dims, pp, pp, pp, pp, pp, pp, pp, pp, 1, ctypes.byref(bad), None) == -1
    assert "hyperparameters" in lib.pinn_last_error().decode()


def test_tuning_cache_file_round_trip(tmp_path):
    """The autotuner's cache written to and merged from a text file; a
    malformed file is rejected and merges nothing (no device needed)."""
    assert lib.pinn_tuning_cache_clear() == 0
    n = ctypes.c_int64(-1)
    assert lib.pinn_tuning_cache_size(ctypes.byref(n)) == 0 and n.value == 0
    good = tmp_path / "tune.txt"
    # a line of the first format (no wide-backward column) and one of the current
    good.write_text("# header\ngfx950 2 1 128 6 16 1 16 1 0.7\ngfx950 1 1 256 8 15 2 32 0 3.25 64\n")
    assert lib.pinn_tuning_cache_load(str(good).encode()) == 0
    assert lib.pinn_tuning_cache_size(ctypes.byref(n)) == 0 and n.value == 2
    out = tmp_path / "out.txt"
    assert lib.pinn_tuning_cache_save(str(out).encode()) == 0
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert sorted(l.split()[:9] for l in lines) == sorted(l.split()[:9] for l in good.read_text().splitlines()[1:])
    assert sorted(l.split()[10] for l in lines) == ["0", "64"]
    for bad_line in ("gfx950 2 1 128 6 16 7 16 1 0.7\n",      # split mode 7 does not exist
                     "gfx950 2 1 128 6 16 1 16 1 0.7 48\n"):  # no 48-point wide backward tiling
        bad = tmp_path / "bad.txt"
        bad.write_text(bad_line)
        assert lib.pinn_tuning_cache_load(str(bad).encode()) == -1
        assert "malformed" in lib.pinn_last_error().decode()
    assert lib.pinn_tuning_cache_size(ctypes.byref(n)) == 0 and n.value == 2
    assert lib.pinn_tuning_cache_load(str(tmp_path / "missing.txt").encode()) == -1
    assert lib.pinn_tuning_cache_clear() == 0
    assert lib.pinn_tuning_cache_size(ctypes.byref(n)) == 0 and n.value == 0


def test_adam_chain_runs():
    """pinn_adam_step takes a chain of layer sizes; the binding splits a
    parameter list into chains: one for a plain MLP, three for the modified
    MLP (U and V encoders, then the chain from the embedding)."""
    from paper_2606_29702_amd.optim import chain_runs
    plain = [(64, 2)] + [(64, 64)] * 5 + [(1, 64)]
    assert chain_runs(plain) == [(0, 7)]
    modified = [(64, 3), (64, 3), (64, 3)] + [(64, 64)] * 5 + [(1, 64)]
    assert chain_runs(modified) == [(0, 1), (1, 2), (2, 9)]
    # every run is a chain and the runs cover every layer once
    for shapes in (plain, modified):
        covered = []
        for a, e in chain_runs(shapes):
            covered += list(range(a, e))
            assert all(shapes[l][1] == shapes[l - 1][0] for l in range(a + 1, e))
        assert covered == list(range(len(shapes)))
