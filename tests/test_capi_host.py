"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and rejects bad
arguments before touching the GPU (these calls return before any HIP call, so they run without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stagcg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stag_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1010_4782_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libstagcg.so is not built: run python -m paper_1010_4782_amd.build")
    return _lib.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("stag_create_lattice", "stag_load_links", "stag_dslash", "stag_cg_solve"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1010_4782_amd import _lib

    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} has no ctypes signature"


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors have the sizes and field offsets a C compiler gives the header's structs."""
    import shutil
    import subprocess

    from paper_1010_4782_amd import _lib

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler on this host")
    mirrors = {"stag_cg_params": _lib.StagParams, "stag_cg_info": _lib.StagInfo, "stag_problem": _lib.StagProblem,
               "stag_shape": _lib.StagShape, "stag_train_params": _lib.StagTrainParams,
               "stag_train_info": _lib.StagTrainInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "stagcg.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname}.{field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for cname, py in mirrors.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for field, _ in py._fields_:
            assert int(got[f"{cname}.{field}"]) == getattr(py, field).offset, f"{cname}.{field}"


def test_params_default(lib):
    from paper_1010_4782_amd import _lib

    p = _lib.default_params()
    assert p.tol == 1e-10 and p.reliable_interval == 50 and p.reliable_delta == 0.1
    assert p.check_interval == 16 and p.max_restarts == 5 and p.prec == 0


@pytest.mark.parametrize("dims", [(3, 4, 4, 4), (4, 4, 4, 0), (4, 4, -2, 4), (4, 4, 4, 5)])
def test_create_lattice_rejects_bad_dims(lib, dims):
    h = C.c_void_p()
    st = lib.stag_create_lattice((C.c_int32 * 4)(*dims), 1, C.byref(h))
    assert st == 1 and not h.value
    assert b"even" in lib.stag_last_error()


def test_create_lattice_rejects_huge_volume(lib):
    h = C.c_void_p()
    assert lib.stag_create_lattice((C.c_int32 * 4)(2048, 2048, 512, 2), 1, C.byref(h)) == 1


def test_null_arguments_are_rejected(lib):
    assert lib.stag_create_lattice(None, 1, None) == 1
    assert lib.stag_destroy_lattice(None) == 1
    assert lib.stag_load_links(None, None, None, -1 / 24, 1, None) == 1
    assert lib.stag_dslash(None, 0, None, None, 1, 0, None) == 1
    assert lib.stag_dslash_slab(None, 0, 0, 2, None, None, 1, 0, None) == 1
    assert lib.stag_apply_m(None, None, None, None, 1, None) == 1
    assert lib.stag_slice_norm2(None, None, 3, 3, 1.0, 0, None, None) == 1
    assert lib.stag_pion_correlator(None, None, 1, 0.1, None, None) == 1
    assert lib.stag_stream_read(None, 32768, None, None) == 1
    assert lib.stag_lattice_info(None, None, None) == 1


def test_batch_argument_validation(lib):
    from paper_1010_4782_amd import _lib

    info = (_lib.StagInfo * 1)()
    prm = _lib.default_params()
    assert lib.stag_cg_solve_batch(0, None, C.byref(prm), info, None) == 1
    assert lib.stag_cg_solve_batch(17, None, C.byref(prm), info, None) == 1
    probs = (_lib.StagProblem * 1)()
    assert lib.stag_cg_solve_batch(1, probs, C.byref(prm), info, None) == 1      # NULL lattice
    prm.tol = -1.0
    assert lib.stag_cg_solve_batch(1, probs, C.byref(prm), info, None) == 1
    assert b"tol" in lib.stag_last_error()


def test_tune_cache_roundtrip(lib, tmp_path):
    """The tuning table loads from and saves to JSON without a GPU; malformed entries are refused."""
    src = tmp_path / "tune.json"
    # an entry without the LDS flag (older files) reads as unstaged
    # (and without the time chunks: 1); a time-streaming entry keeps its chunks
    src.write_text('{\n  "p2:28x28x28x96/1": [256, 1, 1],\n  "p0:8x8x8x8/8": [128, 8],\n'
                   '  "p2c:48x48x48x144/8": [64, 8, 0, 2, 4]\n}\n')
    assert lib.stag_tune_cache_load(str(src).encode()) == 0
    out = tmp_path / "out.json"
    assert lib.stag_tune_cache_save(str(out).encode()) == 0
    text = out.read_text()
    assert '"p2:28x28x28x96/1": [256, 1, 1, 0, 1]' in text and '"p0:8x8x8x8/8": [128, 8, 0, 0, 1]' in text
    assert '"p2c:48x48x48x144/8": [64, 8, 0, 2, 4]' in text
    bad = tmp_path / "bad.json"
    for entry in ("[100, 3]", "[256, 1, 2]", "[64, 1, 0, 3]", "[64, 8, 0, 2, 0]"):
        bad.write_text('{\n  "p0:8x8x8x8/8": %s\n}\n' % entry)
        assert lib.stag_tune_cache_load(str(bad).encode()) == 1, entry
    assert lib.stag_tune_cache_load(str(tmp_path / "missing.json").encode()) == 1
    assert lib.stag_tune_cache_load(None) == 1


def test_shape_arguments_validated(lib):
    assert lib.stag_set_dslash_shape(None, 0, 1, None) == 1
    assert lib.stag_tune_dslash(None, 0, 1, None, None, 0, None, None) == 1


def test_network_arguments_validated(lib):
    h = C.c_void_p()
    assert lib.stag_net_create(None, 4, 8, 0, 0, C.byref(h)) == 1
    assert lib.stag_net_destroy(None) == 1
    assert lib.stag_net_apply(None, None, None, 1, None) == 1
    assert lib.stag_net_num_weights(None, None) == 1
    assert lib.stag_net_train(None, None, None, 1, None, None, None) == 1
