"""The library's host code (argument checks, workspace layout, error paths
of the C-ABI) under AddressSanitizer: nlinv_abi.cpp is rebuilt with the
sanitizer on its host code only, linked with the kernel objects of the normal
build, and a C program drives the host-only entry points and the error paths
that return before any device call.  No GPU is needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "nlinv.h"

static int expect(int got, int want, const char* what) {
  if (got != want) { fprintf(stderr, "%s: got %d, want %d\n", what, got, want); return 1; }
  return 0;
}

int main(void) {
  int bad = 0;
  nlinv_params p;
  size_t ws;
  int32_t R, G, Gc;
  int64_t S, X;
  const int Ns[] = {32, 64, 128, 160, 192, 224};
  for (int i = 0; i < 6; ++i) {
    nlinv_params_default(&p);
    p.N = Ns[i]; p.J = 1 + 9 * i; p.K = 2 * i + 1; p.U = 1 + i; p.batch = 1 + 3 * i;
    bad += expect(nlinv_sizes(&p, &R, &G, &Gc, &S, &X), NLINV_OK, "sizes");
    bad += expect(nlinv_sizes(&p, NULL, NULL, NULL, NULL, NULL), NLINV_OK, "sizes, no outputs");
    bad += expect(nlinv_workspace_size(&p, &ws), NLINV_OK, "workspace");
  }
  /* rejected parameter sets */
  nlinv_params_default(&p); p.N = 100; p.J = 8; p.K = 13;
  bad += expect(nlinv_workspace_size(&p, &ws), NLINV_E_SIZE, "unsupported grid");
  nlinv_params_default(&p); p.N = 64; p.J = 0; p.K = 13;
  bad += expect(nlinv_workspace_size(&p, &ws), NLINV_E_ARG, "J = 0");
  nlinv_params_default(&p); p.N = 64; p.J = 8; p.K = 12;
  bad += expect(nlinv_workspace_size(&p, &ws), NLINV_E_ARG, "even K");
  nlinv_params_default(&p); p.N = 64; p.J = 8; p.K = 13; p.flags = 64;
  bad += expect(nlinv_workspace_size(&p, &ws), NLINV_E_ARG, "unknown flag");
  bad += expect(nlinv_workspace_size(NULL, &ws), NLINV_E_ARG, "NULL params");
  nlinv_params_default(&p); p.N = 64; p.J = 8; p.K = 13; p.col_tile = 2;
  bad += expect(nlinv_workspace_size(&p, &ws), NLINV_E_ARG, "col_tile 2");
  nlinv_params_default(&p); p.N = 64; p.J = 8; p.K = 13; p.G = 448;
  bad += expect(nlinv_workspace_size(&p, &ws), NLINV_E_SIZE, "gamma > 2");
  nlinv_params_default(&p); p.N = 160; p.J = 8; p.K = 13; p.G = 448; p.flags = NLINV_F_CHECK_FINITE;
  bad += expect(nlinv_workspace_size(&p, &ws), NLINV_OK, "gamma 1.4, finiteness check");
  if (!nlinv_last_error(NULL) || strlen(nlinv_last_error(NULL)) == 0) bad += 1;
  /* plan creation fails on the workspace before touching the device */
  nlinv_params_default(&p); p.N = 64; p.J = 8; p.K = 13;
  nlinv_plan plan = NULL;
  bad += expect(nlinv_plan_create(&p, NULL, NULL, 0, &plan), NLINV_E_WORKSPACE, "NULL workspace");
  bad += expect(plan == NULL, 1, "no plan on failure");
  /* every call on a NULL plan is an argument error */
  bad += expect(nlinv_sync(NULL), NLINV_E_ARG, "sync(NULL)");
  bad += expect(nlinv_set_graphs(NULL, 1), NLINV_E_ARG, "set_graphs(NULL)");
  bad += expect(nlinv_set_batch(NULL, 1), NLINV_E_ARG, "set_batch(NULL)");
  bad += expect(nlinv_psf_samples(NULL, NULL, 1, 0), NLINV_E_ARG, "psf_samples(NULL)");
  bad += expect(nlinv_psf_spokes(NULL, NULL, 1, 0), NLINV_E_ARG, "psf_spokes(NULL)");
  bad += expect(nlinv_plan_destroy(NULL), NLINV_E_ARG, "destroy(NULL)");
  /* budget bookkeeping (host-only) */
  size_t used = 1;
  bad += expect(nlinv_set_budget(-1, 0), NLINV_E_ARG, "set_budget(-1)");
  bad += expect(nlinv_set_budget(64, 0), NLINV_E_ARG, "set_budget(64)");
  bad += expect(nlinv_budget_used(0, NULL), NLINV_E_ARG, "budget_used(NULL)");
  bad += expect(nlinv_budget_used(0, &used), NLINV_OK, "budget_used");
  bad += expect(used == 0, 1, "no plans, nothing used");
  bad += expect(nlinv_set_budget(0, 1 << 20), NLINV_OK, "set_budget");
  bad += expect(nlinv_set_budget(0, 0), NLINV_OK, "clear budget");
  /* the static workspace refuses parameters that need more than it holds */
  nlinv_params_default(&p); p.N = 256; p.J = 64; p.K = 21; p.U = 8; p.batch = 4;
  bad += expect(nlinv_plan_workspace_size(&p, &ws), NLINV_OK, "plan_workspace_size");
  bad += expect(ws > NLINV_STATIC_WORKSPACE_BYTES, 1, "oversized for the static workspace");
  plan = NULL;
  bad += expect(nlinv_plan_create_static(&p, NULL, &plan), NLINV_E_WORKSPACE, "create_static oversized");
  bad += expect(plan == NULL, 1, "no static plan on failure");
  bad += expect(nlinv_plan_create_static(&p, NULL, NULL), NLINV_E_ARG, "create_static(NULL out)");
  printf("checks done, %d failed\n", bad);
  return bad != 0;
}
"""


@pytest.mark.skipif(not os.path.exists(CLANG), reason="no ROCm clang")
def test_host_code_under_address_sanitizer(tmp_path):
    import sys
    sys.path.insert(0, ROOT)
    from paper_1701_08361_amd import build as B
    objs = [os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o") for s in B.SOURCES if s != "nlinv_abi.cpp"]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("kernel objects not built")
    abi_o = str(tmp_path / "abi_asan.o")
    host_asan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    r = subprocess.run([B.HIPCC, *B.COMMON, "-x", "hip", "-c", os.path.join(B.CSRC, "nlinv_abi.cpp"),
                        *host_asan, "-o", abi_o], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    lib = str(tmp_path / "libnlinv.so")
    r = subprocess.run([B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", abi_o, *objs,
                        "-Xarch_host", "-shared-libasan", *host_asan, "-o", lib], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    src = tmp_path / "drive.c"
    src.write_text(PROGRAM)
    exe = str(tmp_path / "drive")
    rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    rtdir = os.path.dirname(rt)
    if not os.path.exists(rt):
        rtdir = subprocess.run([CLANG, "-print-runtime-dir"], capture_output=True, text=True).stdout.strip()
    r = subprocess.run([CLANG, "-std=c99", "-Wall", "-Werror", "-fsanitize=address", "-shared-libasan",
                        "-I", os.path.join(ROOT, "include"), str(src), "-L", str(tmp_path), "-lnlinv",
                        f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{rtdir}", "-o", exe], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert "AddressSanitizer" not in run.stderr, run.stderr[-3000:]
    assert run.returncode == 0, (run.returncode, run.stdout, run.stderr[-2000:])
    assert "0 failed" in run.stdout
