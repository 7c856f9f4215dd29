"""The C-ABI library loads and exports every entry point its header declares;
host-side argument validation (no GPU work) behaves as documented."""
import ctypes as ct
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _declared():
    names = set()
    for f in os.listdir(HEADER_DIR):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mhdpic_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1412_1087_amd import mhdpic as M
    if not os.path.exists(M.LIB_PATH):
        from paper_1412_1087_amd import build as B
        B.build()
    return M.lib()


def test_header_declares_the_core_calls():
    names = _declared()
    for n in ("mhdpic_init", "mhdpic_step", "mhdpic_deposit_read", "mhdpic_particles_read",
              "mhdpic_workspace_size", "mhdpic_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1412_1087_amd import mhdpic as M
    for n in _declared():
        assert hasattr(lib, n), f"{n} declared but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", M.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert set(_declared()) <= exported
    assert set(M.EXPORTED) == set(_declared())


def test_workspace_size_validation(lib):
    from paper_1412_1087_amd import mhdpic as M
    b = M.Box(ndim=3, n=(16, 16, 16))
    assert M.workspace_size([b], [1000]) > 0
    with pytest.raises(M.MhdpicError) as e:
        M.workspace_size([M.Box(ndim=4, n=(4, 4, 4))], [10])
    assert e.value.code == M.EINVAL
    raw = M.Box(ndim=2, n=(8, 8)).c_struct()
    raw.n[2] = 2  # 2D boxes must have n[2] = 1
    npart = (ct.c_int64 * 1)(10)
    size = ct.c_size_t()
    assert lib.mhdpic_workspace_size(ct.byref(raw), 1, npart, 0, ct.byref(size)) == M.EINVAL
    with pytest.raises(M.MhdpicError) as e:
        M.workspace_size([M.Box(ndim=3, n=(4096, 4, 4))], [10])
    assert e.value.code == M.ERANGE
    with pytest.raises(M.MhdpicError) as e:
        M.workspace_size([M.Box(ndim=3, n=(8, 8, 8), tile=(5, 5, 5))], [10])
    assert e.value.code == M.ENOTSUP
    with pytest.raises(M.MhdpicError) as e:
        M.workspace_size([M.Box(ndim=2, n=(8, 8)), M.Box(ndim=3, n=(8, 8, 8))], [1, 1])
    assert e.value.code == M.EINVAL
    with pytest.raises(M.MhdpicError) as e:
        M.workspace_size([M.Box(ndim=2, n=(8, 8), C=-1.0)], [1])
    assert e.value.code == M.EINVAL
    with pytest.raises(M.MhdpicError) as e:
        M.workspace_size([M.Box(ndim=2, n=(8, 8), max_move_cells=3)], [1])
    assert e.value.code == M.EINVAL
    with pytest.raises(M.MhdpicError):
        M.workspace_size([b], [-1])
    # precision forms
    assert M.workspace_size([b], [1000], M.FP32_MIXED) < M.workspace_size([b], [1000], M.FP64)


def test_workspace_grows_with_particles(lib):
    from paper_1412_1087_amd import mhdpic as M
    b = M.Box(ndim=2, n=(64, 64))
    s1 = M.workspace_size([b], [10_000])
    s2 = M.workspace_size([b], [20_000])
    # two particle buffers of 64 B/particle (2D, binary64) + the key
    assert s2 - s1 >= 0.99 * 10_000 * (2 * 64 + 4)


def test_null_context_calls_are_rejected(lib):
    from paper_1412_1087_amd import mhdpic as M
    assert lib.mhdpic_step(None, None, None, None, None, 1, None) == M.EINVAL
    assert lib.mhdpic_deposit_read(None, None, 0, None) == M.EINVAL
    assert lib.mhdpic_particles_read(None, None, None, None) == M.EINVAL
    assert lib.mhdpic_check(None, None) == M.EINVAL
    assert lib.mhdpic_destroy(None) == M.OK
    assert b"NULL" in lib.mhdpic_last_error()


def test_tile_shapes_that_exceed_the_lds_are_rejected(lib):
    from paper_1412_1087_amd import mhdpic as M
    b = M.Box(ndim=3, n=(16, 16, 16), tile=(8, 8, 8))
    with pytest.raises(M.MhdpicError) as e:
        M.workspace_size([b], [100], M.FP64)  # 170 KB of LDS in binary64
    assert e.value.code == M.ENOTSUP
    assert M.workspace_size([b], [100], M.FP32_MIXED) > 0
