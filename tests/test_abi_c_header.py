"""The boundary is a plain C ABI: a C99 program that includes include/nlinv.h
compiles without warnings, links against the built library and runs its
host-only entry points (parameter defaults, derived sizes, workspace size,
argument rejection) without a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1701_08361_amd")

PROGRAM = r"""
#include <stdio.h>
#include "nlinv.h"

int main(void) {
  nlinv_params p;
  if (nlinv_params_default(&p) != NLINV_OK) return 10;
  p.N = 160; p.J = 10; p.K = 15; p.U = 5;
  int32_t R, G, Gc;
  int64_t S, X;
  if (nlinv_sizes(&p, &R, &G, &Gc, &S, &X) != NLINV_OK) return 11;
  size_t ws = 0;
  if (nlinv_workspace_size(&p, &ws) != NLINV_OK || ws == 0) return 12;
  printf("%d %d %d %lld %lld %zu\n", (int)R, (int)G, (int)Gc, (long long)S, (long long)X, ws);
  p.K = 14;   /* even spoke counts are rejected */
  if (nlinv_workspace_size(&p, &ws) != NLINV_E_ARG) return 13;
  if (nlinv_last_error(NULL) == NULL) return 14;
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_header_is_c99_and_host_entry_points_run(tmp_path):
    lib = os.path.join(LIBDIR, "libnlinv.so")
    if not os.path.exists(lib):
        pytest.skip("libnlinv.so not built")
    src = tmp_path / "abi.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "abi"
    cc = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                         "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                         "-L", LIBDIR, "-lnlinv", f"-Wl,-rpath,{LIBDIR}"],
                        capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, (run.returncode, run.stderr)
    R, G, Gc, S, X, ws = run.stdout.split()
    # 160 px: R = 160, G = 320, G_c = 80, S = 15 * 320, X = 160^2 + 10 * 80^2
    assert (int(R), int(G), int(Gc), int(S), int(X)) == (160, 320, 80, 4800, 89600)
    assert int(ws) > 0
