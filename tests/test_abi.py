"""The C-ABI library loads and exports every function include/bounce.h declares;
the ctypes structures have the C layout (checked against gcc on the header).
No GPU work is done here."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bounce.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bounce_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    from paper_2002_07109_amd import _abi
    assert _declared() == sorted(_abi.SIGNATURES)


def test_library_exports_every_symbol():
    from paper_2002_07109_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libbounce.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (bounce_[a-z_]+)$", out, flags=re.M))
    missing = set(_declared()) - exported
    assert not missing, missing
    L = _abi.load()
    for name in _declared():
        assert getattr(L, name) is not None


def test_struct_layout_matches_c(tmp_path):
    from paper_2002_07109_amd import _abi
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "bounce.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(bounce_params),'
                   ' sizeof(bounce_system), sizeof(bounce_counters), sizeof(bounce_event),'
                   ' offsetof(bounce_params, dt), offsetof(bounce_system, n_types)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    exp = [C.sizeof(_abi.bounce_params), C.sizeof(_abi.bounce_system),
           C.sizeof(_abi.bounce_counters), C.sizeof(_abi.bounce_event),
           _abi.bounce_params.dt.offset, _abi.bounce_system.n_types.offset]
    assert got == exp


def test_argument_errors_need_no_gpu():
    from paper_2002_07109_amd import _abi, make_params
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libbounce.so not built")
    L = _abi.load()
    ctx = C.c_void_p()
    bad = make_params(dt=-1.0)
    assert L.bounce_create(C.byref(bad), C.byref(ctx)) == _abi.E_ARG
    good = make_params()
    assert L.bounce_create(C.byref(good), C.byref(ctx)) == _abi.OK
    assert L.bounce_step(ctx, 1) == _abi.E_STATE          # no system bound yet
    nb = C.c_uint64()
    assert L.bounce_workspace_size(ctx, C.byref(nb)) == _abi.E_STATE
    assert L.bounce_status_string(_abi.E_SKIN).decode().startswith("an atom moved")
    L.bounce_destroy(ctx)
    # mesh parameters: powers of two in [8, 512], order 4..6, periodic, and a
    # RESPA outer step that divides the rebuild interval
    for kw in (dict(pme_grid=(24, 32, 32)), dict(pme_grid=(4, 4, 4)), dict(pme_grid=(1024, 8, 8)),
               dict(pme_grid=(32, 32, 32), pme_order=3), dict(pme_grid=(32, 32, 32), pme_order=7),
               dict(pme_grid=(32, 32, 32), periodic=0),
               dict(pme_grid=(32, 32, 32), respa_m=3, rebuild_interval=10),
               dict(pme_grid=(32, 32, 32), respa_m=-1), dict(respa_outer=1, respa_m=0),
               dict(respa_outer=2, respa_m=2), dict(respa_outer=1, respa_m=3, rebuild_interval=10)):
        p = make_params(**kw)
        assert L.bounce_create(C.byref(p), C.byref(ctx)) == _abi.E_ARG, kw
    p = make_params(pme_grid=(16, 32, 64), pme_order=6, respa_m=5, rebuild_interval=10)
    assert L.bounce_create(C.byref(p), C.byref(ctx)) == _abi.OK
    L.bounce_destroy(ctx)
    p = make_params(periodic=0, respa_m=2, respa_outer=1)        # outer pair force, no mesh
    assert L.bounce_create(C.byref(p), C.byref(ctx)) == _abi.OK
    L.bounce_destroy(ctx)
    # launch structure and partner search: persistent 0/1; cluster tiles of 4 or 8
    # atoms, FP32 pair arithmetic only
    for kw in (dict(persistent=2), dict(pair_kernel=6), dict(pair_kernel=4, pair_precision=1)):
        p = make_params(**kw)
        assert L.bounce_create(C.byref(p), C.byref(ctx)) == _abi.E_ARG, kw
    for kw in (dict(persistent=1), dict(pair_kernel=8), dict(pair_kernel=4, persistent=1)):
        p = make_params(**kw)
        assert L.bounce_create(C.byref(p), C.byref(ctx)) == _abi.OK, kw
        L.bounce_destroy(ctx)


def test_missing_library_fails_loudly(tmp_path):
    """Without libbounce.so the package refuses to run: there is no fallback."""
    import paper_2002_07109_amd._abi as abi
    with pytest.raises(ImportError):
        abi.load(str(tmp_path / "libbounce.so"))
