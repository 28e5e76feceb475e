"""The C-ABI used from C alone: a C program (HIP runtime API and nlinv.h, no
PyTorch) allocates the workspace, builds the PSF kernels, grids and
reconstructs a two-frame series with temporal regularisation.  Its images
equal, bit for bit, those of the Python binding making the same calls."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1701_08361_amd import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1701_08361_amd")

PROGRAM = r"""
#include <stdio.h>
#include <stdlib.h>
#include <hip/hip_runtime_api.h>
#include "nlinv.h"

#define CK(x) do { int e_ = (x); if (e_) { fprintf(stderr, "%s: %d %s\n", #x, e_, \
                   nlinv_last_error(plan)); return 1; } } while (0)
#define HK(x) do { if ((x) != hipSuccess) { fprintf(stderr, "%s failed\n", #x); return 2; } } while (0)

static void* slurp(const char* path, size_t bytes) {
  void* p = malloc(bytes);
  FILE* f = fopen(path, "rb");
  if (!f || fread(p, 1, bytes, f) != bytes) { free(p); p = NULL; }
  if (f) fclose(f);
  return p;
}

int main(int argc, char** argv) {
  if (argc != 10) return 3;
  const int N = atoi(argv[1]), J = atoi(argv[2]), K = atoi(argv[3]), U = atoi(argv[4]);
  const int M = atoi(argv[5]), C = atoi(argv[6]), F = atoi(argv[7]);
  nlinv_plan plan = NULL;
  nlinv_params p;
  nlinv_params_default(&p);
  p.N = N; p.J = J; p.K = K; p.U = U; p.newton = M; p.cg = C;
  int32_t R, G, Gc; int64_t S, X;
  CK(nlinv_sizes(&p, &R, &G, &Gc, &S, &X));
  const size_t tb = (size_t)K * (S / K) * 2 * sizeof(float), yb = (size_t)J * S * sizeof(nlinv_c64);
  float* h_traj = (float*)slurp(argv[8], F * tb);
  nlinv_c64* h_y = (nlinv_c64*)slurp(argv[9], F * yb);
  if (!h_traj || !h_y) return 4;
  size_t bytes;
  CK(nlinv_workspace_size(&p, &bytes));
  void *ws, *d_traj, *d_y, *d_z, *d_x[2], *d_img;
  HK(hipMalloc(&ws, bytes));
  HK(hipMalloc(&d_traj, F * tb));
  HK(hipMalloc(&d_y, F * yb));
  HK(hipMalloc(&d_z, (size_t)J * R * R * sizeof(nlinv_c64)));
  HK(hipMalloc(&d_x[0], X * sizeof(nlinv_c64)));
  HK(hipMalloc(&d_x[1], X * sizeof(nlinv_c64)));
  HK(hipMalloc(&d_img, (size_t)R * R * sizeof(float)));
  HK(hipMemcpy(d_traj, h_traj, F * tb, hipMemcpyHostToDevice));
  HK(hipMemcpy(d_y, h_y, F * yb, hipMemcpyHostToDevice));
  CK(nlinv_plan_create(&p, NULL, ws, bytes, &plan));
  for (int t = 0; t < U && t < F; ++t) CK(nlinv_psf(plan, (const float*)((char*)d_traj + t * tb), t));
  float* img = (float*)malloc((size_t)R * R * sizeof(float));
  for (int n = 0; n < F; ++n) {
    const int32_t turn = n % U;
    CK(nlinv_grid(plan, (const float*)((char*)d_traj + n * tb), (const nlinv_c64*)((char*)d_y + n * yb),
                  &turn, (nlinv_c64*)d_z));
    CK(nlinv_reconstruct(plan, (const nlinv_c64*)d_z, &turn, n ? (const nlinv_c64*)d_x[(n - 1) & 1] : NULL,
                         (nlinv_c64*)d_x[n & 1], n ? 2 : 1, (float*)d_img, NULL));
    CK(nlinv_sync(plan));
    HK(hipMemcpy(img, d_img, (size_t)R * R * sizeof(float), hipMemcpyDeviceToHost));
    fwrite(img, sizeof(float), (size_t)R * R, stdout);
  }
  CK(nlinv_plan_destroy(plan));
  return 0;
}
"""


def build_program(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "recon.c"
    src.write_text(PROGRAM)
    exe = str(tmp_path / "recon")
    r = subprocess.run([cc, "-std=c99", "-O1", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                        "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include", str(src),
                        "-L", LIBDIR, "-lnlinv", "-L", "/opt/rocm/lib", "-lamdhip64",
                        f"-Wl,-rpath,{LIBDIR}", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def test_c_program_matches_binding(tmp_path):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1701_08361_amd import nlinv
    nlinv.load()
    N, J, K, U, M, C, F = 32, 4, 5, 2, 3, 4, 2
    print(f"[case] C program N={N} J={J} K={K} U={U} M={M} C={C} frames={F}", flush=True)
    ser = synth.real_time_series(seed=31, N=N, J=J, J_phys=6, K=K, U=U, frames=F)
    assert [int(t) for t in ser.turn] == [n % U for n in range(F)]
    (tmp_path / "traj.bin").write_bytes(np.ascontiguousarray(ser.traj, np.float32).tobytes())
    (tmp_path / "y.bin").write_bytes(np.ascontiguousarray(ser.y, np.complex64).tobytes())
    exe = build_program(tmp_path)
    run = subprocess.run([exe, *map(str, (N, J, K, U, M, C, F)), str(tmp_path / "traj.bin"),
                          str(tmp_path / "y.bin")], capture_output=True, timeout=120)
    assert run.returncode == 0, run.stderr.decode()[-2000:]
    imgs_c = np.frombuffer(run.stdout, np.float32).reshape(F, N, N)
    plan = nlinv.Plan(N, J, K, U=U, newton=M, cg=C)
    traj = torch.from_numpy(ser.traj).cuda()
    y = torch.from_numpy(ser.y).cuda()
    for t in range(U):
        plan.psf(traj[t].contiguous(), t)
    prev = None
    for n in range(F):
        z = plan.grid(traj[n:n + 1], y[n:n + 1], turns=[n % U])
        x, img, _ = plan.reconstruct(z, [n % U], xprev=prev, init=2 if n else 1, want_img=True)
        prev = x
        assert np.array_equal(img.cpu().numpy()[0], imgs_c[n]), n
    assert np.isfinite(imgs_c).all() and imgs_c.max() > 0
