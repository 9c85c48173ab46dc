"""The C-ABI library loads and exports every function include/psf.h declares
(no GPU needed: nothing is computed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "psf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("psf_create_table", "psf_insert_samples", "psf_temporal_update", "psf_query",
                     "psf_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2005_07547_amd import psf
    lib = psf.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(n for n, _, _ in psf.EXPORTS) == _declared()


def test_host_side_validation_without_gpu():
    from paper_2005_07547_amd import psf
    lib = psf.load()
    good = psf.make_config(log2_slots=20)
    assert lib.psf_table_bytes(ctypes.byref(good)) >= (1 << 20) * 48
    bad = psf.make_config(log2_slots=31)
    assert lib.psf_table_bytes(ctypes.byref(bad)) == 0
    assert b"log2_slots" in lib.psf_last_error()
    assert lib.psf_table_bytes(None) == 0
    h = ctypes.c_void_p()
    assert lib.psf_create_table(None, None, 0, None, ctypes.byref(h)) == psf.PSF_INVALID_ARGUMENT
    assert lib.psf_destroy(None) == psf.PSF_OK
    assert lib.psf_iterate_batch(None, None, 0, None) == psf.PSF_OK
    assert lib.psf_iterate_batch(None, None, 2, None) == psf.PSF_INVALID_ARGUMENT
    assert lib.psf_batch_destroy(None) == psf.PSF_OK
    assert lib.psf_estimate(None, None, None, 4, 0, 1.0, None, None, None) == psf.PSF_INVALID_ARGUMENT
    assert lib.psf_version().startswith(b"psf")


def test_table_without_accumulators_bytes():
    """PSF_FLAG_NO_ACCUMULATORS leaves out the 16-byte per-slot frame
    accumulator (and the 8-byte pending squared-luminance sum of a variance
    table); it needs the RGB payload and the partitioned strategy."""
    from paper_2005_07547_amd import psf
    lib = psf.load()

    def nbytes(**kw):
        return lib.psf_table_bytes(ctypes.byref(psf.make_config(**kw)))

    S = 1 << 20
    plain = nbytes(log2_slots=20, max_batch=1 << 18)
    lean = nbytes(log2_slots=20, max_batch=1 << 18, flags=psf.PSF_FLAG_NO_ACCUMULATORS)
    assert plain - lean == S * 16
    var = psf.PSF_FLAG_TRACK_VARIANCE
    assert (nbytes(log2_slots=20, max_batch=1 << 18, flags=var)
            - nbytes(log2_slots=20, max_batch=1 << 18, flags=var | psf.PSF_FLAG_NO_ACCUMULATORS)) == S * 24
    assert nbytes(log2_slots=20, flags=psf.PSF_FLAG_NO_ACCUMULATORS, insert_mode=psf.PSF_INSERT_DIRECT) == 0
    assert b"partitioned" in lib.psf_last_error()
    assert nbytes(log2_slots=20, flags=psf.PSF_FLAG_NO_ACCUMULATORS, payload=psf.PSF_PAYLOAD_SH2_YCOCG,
                  insert_mode=psf.PSF_INSERT_DIRECT) == 0
    # more partitions than the partitioned strategy takes (2^28 slots of 2^11)
    assert nbytes(log2_slots=28, part_log2=11, flags=psf.PSF_FLAG_NO_ACCUMULATORS) == 0
    assert b"partitioned strategy" in lib.psf_last_error()
    assert nbytes(log2_slots=20, flags=32) == 0


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structures against the C layouts of include/psf.h,
    compiled by the host C compiler."""
    import shutil
    import subprocess
    from paper_2005_07547_amd import psf
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    structs = {"psf_config": psf.psf_config, "psf_records": psf.psf_records,
               "psf_queries": psf.psf_queries, "psf_stats": psf.psf_stats,
               "psf_session": psf.psf_session, "psf_estimate_args": psf.psf_estimate_args,
               "psf_step_args": psf.psf_step_args, "psf_prim": psf.psf_prim, "psf_camera": psf.psf_camera,
               "psf_path_params": psf.psf_path_params, "psf_path_out": psf.psf_path_out}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "psf.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        k, v = line.rsplit(" ", 1)
        got[k] = int(v)
    for name, cls in structs.items():
        assert got[f"{name} size"] == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert got[f"{name}.{fname}"] == getattr(cls, fname).offset, (name, fname)
