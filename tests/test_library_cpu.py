"""The C interface library builds for gfx950, loads, exports every declared
entry point, and rejects bad arguments before touching a device (CPU only)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(hjg_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2605_18566_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2605_18566_amd.build import build
        build()
    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
    from paper_2605_18566_amd import _lib
    assert {s[0] for s in _lib.SIGNATURES} == set(names)


def test_struct_layout_matches_header(lib, tmp_path):
    import shutil
    import subprocess
    from paper_2605_18566_amd import _lib
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hjg.h"\nint main(){printf("%zu %zu %zu %zu\\n",'
                   'sizeof(hjg_problem), offsetof(hjg_problem, datum_aux), offsetof(hjg_problem, seed),'
                   'offsetof(hjg_problem, problem_id));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [C.sizeof(_lib.Problem), _lib.Problem.datum_aux.offset, _lib.Problem.seed.offset,
                   _lib.Problem.problem_id.offset]
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hjg.h"\nint main(){printf("%zu %zu %zu %zu\\n",'
                   'sizeof(hjg_budget), offsetof(hjg_budget, C2), offsetof(hjg_budget, N),'
                   'offsetof(hjg_budget, delta));return 0;}\n')
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [C.sizeof(_lib.Budget), _lib.Budget.C2.offset, _lib.Budget.N.offset, _lib.Budget.delta.offset]


def test_error_budget_matches_oracle(lib):
    # host arithmetic only: no device needed
    import numpy as np
    from oracle import certify as oc
    from paper_2605_18566_amd import error_budget
    args = (1.5, 0.7, 5, 2.0, 65536, 0.01, 3e-3, 0.8, 0.02)
    np.testing.assert_allclose(error_budget(*args), oc.error_budget(*args), rtol=1e-15)
    from paper_2605_18566_amd import _lib
    with pytest.raises(_lib.HJGError):
        error_budget(1.0, 0.5, 3, 1.0, 100, 1.5)


def test_version_and_error_paths_without_device(lib):
    from paper_2605_18566_amd import _lib
    assert lib.hjg_version().startswith(b"hjg")
    assert lib.hjg_philox4x32_10(0, 0, 0, 0, 0, None, None) == _lib.HJG_OK          # G = 0: no launch
    assert lib.hjg_philox4x32_10(0, 0, 0, 0, -1, None, None) == _lib.HJG_EINVAL
    p = _lib.Problem()
    p.n, p.nu, p.c_min, p.c_max = 2, 0.05, 0.01, 1e4
    rc = lib.hjg_value_grad(None, C.byref(p), 4, None, 0.5, 16, 0, 0, None, None, None, None, None, 0, None)
    assert rc == _lib.HJG_EINVAL and b"context" in lib.hjg_last_error()
    rc = lib.hjg_picard_sweep(None, C.byref(p), 4, None, 0.5, 16, 1, 0.0, 0, None, None, None, None, None, None,
                              None, None, None, None)
    assert rc == _lib.HJG_EINVAL
    rc = lib.hjg_surrogate_tube_step(None, None, C.byref(p), 4, None, 0.0, 0.1, 16, 1, 0.0, 0, None, None, None,
                                     None, None, None, None)
    assert rc == _lib.HJG_EINVAL and b"surrogate" in lib.hjg_last_error()
    h = C.c_void_p()
    assert lib.hjg_surrogate_load(None, b"/nonexistent/x", C.byref(h)) == _lib.HJG_EINVAL
    assert lib.hjg_surrogate_save(None, b"/nonexistent/x") == _lib.HJG_EINVAL
    assert lib.hjg_tuning_save(None, b"/nonexistent/x") == _lib.HJG_EINVAL
    assert lib.hjg_tuning_load(None, b"/nonexistent/x") == _lib.HJG_EINVAL
    # obstacle projection: every check runs before any device work
    assert lib.hjg_avoid_project(None, 4, None, None, None, None, None) == _lib.HJG_EINVAL
    ob = _lib.Problem()
    ob.n, ob.nu, ob.c_min, ob.c_max = 2, 0.05, 0.01, 1e4
    ob.datum = _lib.DATUMS["ball"]
    ob.datum_p[0], ob.datum_p[1] = 2.0, 0.5
    assert lib.hjg_avoid_project(C.byref(ob), -1, None, None, None, None, None) == _lib.HJG_EINVAL
    assert lib.hjg_avoid_project(C.byref(ob), 0, None, None, None, None, None) == _lib.HJG_OK
    assert lib.hjg_avoid_project(C.byref(ob), 4, None, None, None, None, None) == _lib.HJG_EINVAL
    assert b"required" in lib.hjg_last_error()
    ob.datum = _lib.DATUMS["disc_union"]                 # needs its centres
    ob.datum_p[0], ob.datum_p[1] = 0.5, 2.0
    assert lib.hjg_avoid_project(C.byref(ob), 0, None, None, None, None, None) == _lib.HJG_EINVAL
    # only n and the datum fields are checked: a 48-dimensional capture set with
    # fields a sweep would reject (fresh draws at n = 48, nu = NaN) is accepted
    ob.n, ob.datum, ob.sample_mode, ob.nu = 48, _lib.DATUMS["capture"], 0, float("nan")
    ob.datum_p[0] = 0.4
    assert lib.hjg_avoid_project(C.byref(ob), 0, None, None, None, None, None) == _lib.HJG_OK
    assert lib.hjg_value_grad(None, C.byref(ob), 0, None, 0.5, 16, 0, 0, None, None, None, None, None, 0,
                              None) == _lib.HJG_EINVAL
    lib.hjg_ctx_destroy(None)


def test_kernels_are_gfx950_code_objects(lib):
    from paper_2605_18566_amd import _lib
    blob = open(_lib.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2605_18566_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        _lib.lib()


def test_topology_events_match_oracle(lib):
    # host arithmetic only
    import numpy as np
    from oracle import topology as ot
    from paper_2605_18566_amd import topology_events
    rng = np.random.default_rng(3)
    for _ in range(20):
        T = int(rng.integers(1, 30))
        ncomp = rng.integers(0, 4, T)
        beta1 = rng.integers(0, 3, T) * rng.integers(0, 2, T)
        chi = ncomp - beta1
        np.testing.assert_array_equal(topology_events(chi, beta1, ncomp), ot.events(chi, beta1, ncomp))
