"""The C-ABI library loads, exports every function include/tfstat.h declares,
and the Python binding's struct layouts match the header's (checked by
compiling the header with gcc).  Only argument validation that returns
before any device call is exercised here."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1805_05652_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tfstat.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(tfstat_[A-Za-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    names = _declared_functions()
    assert "tfstat_fmap" in names and "tfstat_submit" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_abi.SIGNATURES), set(names) ^ set(_abi.SIGNATURES)


def test_struct_layouts_match_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "tfstat.h"
#define F(s, f) printf(#s "." #f " %zu\n", offsetof(s, f))
int main(void) {
  printf("tfstat_window %zu\n", sizeof(tfstat_window));
  F(tfstat_window, type); F(tfstat_window, n_t0); F(tfstat_window, n_tau);
  F(tfstat_window, t0_min); F(tfstat_window, dt0); F(tfstat_window, tau_min);
  F(tfstat_window, dtau); F(tfstat_window, t0_list); F(tfstat_window, tau_list);
  F(tfstat_window, shape); F(tfstat_window, n_shape); F(tfstat_window, support_num);
  F(tfstat_window, support_den); F(tfstat_window, reserved2);
  printf("tfstat_atoms_desc %zu\n", sizeof(tfstat_atoms_desc));
  F(tfstat_atoms_desc, n_sft); F(tfstat_atoms_desc, n_bins); F(tfstat_atoms_desc, t_sft);
  F(tfstat_atoms_desc, timestamps); F(tfstat_atoms_desc, a2); F(tfstat_atoms_desc, fb);
  printf("tfstat_bin_result %zu\n", sizeof(tfstat_bin_result));
  F(tfstat_bin_result, max2F); F(tfstat_bin_result, logB); F(tfstat_bin_result, t0);
  F(tfstat_bin_result, tau); F(tfstat_bin_result, m); F(tfstat_bin_result, n);
  printf("tfstat_batch_stats %zu\n", sizeof(tfstat_batch_stats));
  F(tfstat_batch_stats, variant); F(tfstat_batch_stats, groups); F(tfstat_batch_stats, n_tiles);
  F(tfstat_batch_stats, n_results); F(tfstat_batch_stats, tune_ms); F(tfstat_batch_stats, last_ms);
  F(tfstat_batch_stats, last_fused_ms);
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), "-o", str(exe), str(prog)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    py = {"tfstat_window": _abi.Window, "tfstat_atoms_desc": _abi.AtomsDesc,
          "tfstat_bin_result": _abi.BinResult, "tfstat_batch_stats": _abi.BatchStats}
    for key, val in got.items():
        if "." in key:
            s, f = key.split(".")
            assert getattr(py[s], f).offset == int(val), key
        else:
            assert ctypes.sizeof(py[key]) == int(val), key


def test_argument_validation_without_device():
    lib = _abi.load()
    assert lib.tfstat_version().startswith(b"tfstat")
    # null output / null context are rejected before any device call
    assert lib.tfstat_ctx_create(0, None, 1 << 30, None, None) == _abi.E_INVAL
    assert b"null" in lib.tfstat_last_error()
    out = ctypes.c_void_p()
    assert lib.tfstat_ctx_create(0, ctypes.c_void_p(4096 + 8), 1 << 30, None,
                                 ctypes.byref(out)) == _abi.E_INVAL
    assert b"aligned" in lib.tfstat_last_error()
    assert lib.tfstat_ctx_destroy(None) == _abi.E_INVAL
    assert lib.tfstat_fmap(None, 1, None, 1, None, None) == _abi.E_INVAL
    assert lib.tfstat_poll(None, 1, None, None) == _abi.E_INVAL
    assert lib.tfstat_profile_read(None, 0, None, None) == _abi.E_INVAL


def test_errors_raise_typed_exception():
    with pytest.raises(_abi.TfstatError) as e:
        _abi.check(_abi.load().tfstat_cancel(None, 3))
    assert e.value.code == _abi.E_INVAL
